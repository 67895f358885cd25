// Gram build over the rows of a data matrix X (D x N, samples as columns):
//   A_ij = scale * sum_k op(X_ik, X_jk)
// op min1/min2: the min-covariance of eq. (5); op dot: the covariance of eq. (2).
//
// Upper-triangle 64 x 64 output tiles, one per block of 256 threads, each thread
// a 4 x 4 register tile.  X is streamed through LDS in slabs of 32 samples
// (transposed so a thread reads its 4 rows and 4 columns as two 16-byte LDS
// reads per sample), double-buffered through registers.  Terms are accumulated
// in float32 within a run of 256 samples and in float64 across runs.  The
// min forms use one xor, one med3 and one add per term on the vector ALU; the
// dot form uses one fused multiply-add.
#include "common.h"

namespace mapi {

constexpr int GT = 64;          // tile edge
constexpr int GKS = 32;         // samples per LDS slab
constexpr int GPAD = 4;         // LDS row padding (floats)
constexpr int GFLUSH = 256;     // samples per float32 run

__device__ __forceinline__ void tile_coords(int b, int T, int* ti, int* tj) {
  int i = 0;
  while (b >= T - i) {
    b -= T - i;
    ++i;
  }
  *ti = i;
  *tj = i + b;
}

template <int OP>
__global__ void __launch_bounds__(256)
k_gram(const float* __restrict__ X, int D, int64_t N, int64_t ldx, double scale, float* __restrict__ A, int64_t lda) {
  __shared__ float4 lds4[2 * 2 * GKS * (GT + GPAD) / 4];
  float* lds = reinterpret_cast<float*>(lds4);
  const int T = (D + GT - 1) / GT;
  int ti, tj;
  tile_coords(blockIdx.x, T, &ti, &tj);
  const int i0 = ti * GT, j0 = tj * GT;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;

  // loader mapping: 8 threads per row, 4 consecutive samples each; 2 passes of 32 rows
  const int lrow = tid >> 3, lk = (tid & 7) * 4;

  auto slab = [&](int buf, int m) -> float* { return lds + (buf * 2 + m) * GKS * (GT + GPAD); };

  float4 pre[2][2];   // [matrix][pass]
  auto load_slab = [&](int64_t k0) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int base = m ? j0 : i0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = base + lrow + 32 * h;
        const int64_t k = k0 + lk;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (r < D) {
          const float* src = X + (int64_t)r * ldx + k;
          if (k + 3 < N) {
            v = *reinterpret_cast<const float4*>(src);
          } else {
            if (k + 0 < N) v.x = src[0];
            if (k + 1 < N) v.y = src[1];
            if (k + 2 < N) v.z = src[2];
          }
        }
        pre[m][h] = v;
      }
    }
  };
  auto store_slab = [&](int buf) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      float* s = slab(buf, m);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = lrow + 32 * h;
        s[(lk + 0) * (GT + GPAD) + r] = pre[m][h].x;
        s[(lk + 1) * (GT + GPAD) + r] = pre[m][h].y;
        s[(lk + 2) * (GT + GPAD) + r] = pre[m][h].z;
        s[(lk + 3) * (GT + GPAD) + r] = pre[m][h].w;
      }
    }
  };

  float accf[4][4];
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      accf[a][b] = 0.0f;
      acc[a][b] = 0.0;
    }

  const int64_t nslabs = (N + GKS - 1) / GKS;
  load_slab(0);
  store_slab(0);
  __syncthreads();
  for (int64_t sidx = 0; sidx < nslabs; ++sidx) {
    const int buf = (int)(sidx & 1);
    if (sidx + 1 < nslabs) load_slab((sidx + 1) * GKS);
    const float* si = slab(buf, 0);
    const float* sj = slab(buf, 1);
#pragma unroll 8
    for (int k = 0; k < GKS; ++k) {
      const float4 av = *reinterpret_cast<const float4*>(si + k * (GT + GPAD) + ty * 4);
      const float4 bv = *reinterpret_cast<const float4*>(sj + k * (GT + GPAD) + tx * 4);
      const float a[4] = {av.x, av.y, av.z, av.w};
      const float b[4] = {bv.x, bv.y, bv.z, bv.w};
      uint32_t sb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) sb[q] = sign_bit(b[q]);
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) accf[p][q] = op_acc<OP>(accf[p][q], a[p], b[q], sb[q]);
    }
    if (((sidx + 1) * GKS) % GFLUSH == 0 || sidx + 1 == nslabs) {
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc[p][q] += (double)accf[p][q];
          accf[p][q] = 0.0f;
        }
    }
    if (sidx + 1 < nslabs) {
      store_slab(buf ^ 1);
      __syncthreads();
    }
  }

  // epilogue: tile (i, j) and, off the diagonal, its mirror (j, i)
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int i = i0 + ty * 4 + p;
    if (i >= D) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + tx * 4 + q;
      if (j < D) A[(int64_t)i * lda + j] = (float)(scale * acc[p][q]);
    }
  }
  if (ti != tj) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + tx * 4 + q;
      if (j >= D) continue;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int i = i0 + ty * 4 + p;
        if (i < D) A[(int64_t)j * lda + i] = (float)(scale * acc[p][q]);
      }
    }
  }
}

hipError_t launch_gram(const float* X, int64_t D, int64_t N, int64_t ldx, double scale, int op, float* A, int64_t lda,
                       double* acc64, hipStream_t s) {
  (void)acc64;
  const int T = (int)((D + GT - 1) / GT);
  const int blocks = T * (T + 1) / 2;
  switch (op) {
    case MAPI_OP_MIN1:
      hipLaunchKernelGGL(k_gram<MAPI_OP_MIN1>, dim3(blocks), dim3(256), 0, s, X, (int)D, N, ldx, scale, A, lda);
      break;
    case MAPI_OP_MIN2:
      hipLaunchKernelGGL(k_gram<MAPI_OP_MIN2>, dim3(blocks), dim3(256), 0, s, X, (int)D, N, ldx, scale, A, lda);
      break;
    case MAPI_OP_DOT:
      hipLaunchKernelGGL(k_gram<MAPI_OP_DOT>, dim3(blocks), dim3(256), 0, s, X, (int)D, N, ldx, scale, A, lda);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- deflation
// Vector i is extracted from (I - P P^T) A = A - P Q with Q = P^T A (P
// orthonormal, float64).  Q gains one row per extracted vector.

// q_j = sum_i p_i A_ij for one new column p of P: column sums of a row-weighted
// A, reduced over row chunks into `qpart` and then in a fixed order.
constexpr int QCH = 64;   // row chunks

__global__ void __launch_bounds__(256)
k_deflate_qpart(const float* __restrict__ A, int64_t D, int64_t lda, const double* __restrict__ p,
                double* __restrict__ qpart) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int chunk = blockIdx.y;
  const int64_t rows = (D + QCH - 1) / QCH;
  const int64_t r0 = chunk * rows, r1 = min(D, r0 + rows);
  if (j >= D) return;
  double s = 0.0;
  for (int64_t i = r0; i < r1; ++i) s += p[i] * (double)A[i * lda + j];
  qpart[(int64_t)chunk * D + j] = s;
}

__global__ void k_deflate_qsum(const double* __restrict__ qpart, int64_t D, double* __restrict__ q) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= D) return;
  double s = 0.0;
  for (int c = 0; c < QCH; ++c) s += qpart[(int64_t)c * D + j];
  q[j] = s;
}

// out_ij = fl32(A_ij - sum_l P_il Q_lj), float64 arithmetic.  P: D x k column-major; Q: k x D row-major.
__global__ void __launch_bounds__(256)
k_deflate_apply(const float* __restrict__ A, int64_t D, int64_t lda, const double* __restrict__ P,
                const double* __restrict__ Q, int k, float* __restrict__ out, int64_t ldo) {
  const int64_t i = blockIdx.y;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < D; j += (int64_t)gridDim.x * blockDim.x) {
    double v = (double)A[i * lda + j];
    for (int l = 0; l < k; ++l) v -= P[(int64_t)l * D + i] * Q[(int64_t)l * D + j];
    out[i * ldo + j] = (float)v;
  }
}

// Append w to P: p = w / ||w||_2, then modified Gram-Schmidt against the k
// existing columns, then normalise again; writes P[:, k] (float64) and p_out (float32).
__global__ void __launch_bounds__(1024)
k_mgs_append(double* __restrict__ P, int64_t D, int k, const float* __restrict__ w, float* __restrict__ p_out) {
  __shared__ double sh[16];
  double* pk = P + (int64_t)k * D;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < D; i += blockDim.x) {
    const double v = (double)w[i];
    pk[i] = v;
    s += v * v;
  }
  s = block_sum_f64(s, sh);
  double inv = 1.0 / sqrt(s);
  for (int64_t i = threadIdx.x; i < D; i += blockDim.x) pk[i] *= inv;
  __syncthreads();
  for (int l = 0; l < k; ++l) {
    const double* pl = P + (int64_t)l * D;
    double d = 0.0;
    for (int64_t i = threadIdx.x; i < D; i += blockDim.x) d += pl[i] * pk[i];
    d = block_sum_f64(d, sh);
    for (int64_t i = threadIdx.x; i < D; i += blockDim.x) pk[i] -= d * pl[i];
    __syncthreads();
  }
  s = 0.0;
  for (int64_t i = threadIdx.x; i < D; i += blockDim.x) s += pk[i] * pk[i];
  s = block_sum_f64(s, sh);
  inv = 1.0 / sqrt(s);
  for (int64_t i = threadIdx.x; i < D; i += blockDim.x) {
    pk[i] *= inv;
    p_out[i] = (float)pk[i];
  }
}

hipError_t launch_deflate_q(const float* A, int64_t D, int64_t lda, const double* p, double* q, double* qpart,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_deflate_qpart, dim3((unsigned)((D + 255) / 256), QCH), dim3(256), 0, s, A, D, lda, p, qpart);
  hipLaunchKernelGGL(k_deflate_qsum, dim3((unsigned)((D + 255) / 256)), dim3(256), 0, s, qpart, D, q);
  return hipGetLastError();
}

hipError_t launch_deflate_apply(const float* A, int64_t D, int64_t lda, const double* P, const double* Q, int k,
                                float* out, int64_t ldo, hipStream_t s) {
  const unsigned gx = (unsigned)((D + 255) / 256 < 16 ? (D + 255) / 256 : 16);
  hipLaunchKernelGGL(k_deflate_apply, dim3(gx, (unsigned)D), dim3(256), 0, s, A, D, lda, P, Q, k, out, ldo);
  return hipGetLastError();
}

hipError_t launch_mgs_append(double* P, int64_t D, int k, const float* w, float* p_out, hipStream_t s) {
  hipLaunchKernelGGL(k_mgs_append, dim3(1), dim3(1024), 0, s, P, D, k, w, p_out);
  return hipGetLastError();
}

int deflate_qpart_count() { return QCH; }

}  // namespace mapi
