// Mini-batch MAPI with momentum (Algorithm 3, Sec. 3.2): one block per run
// iterates, for t = 0 .. T-1 with the batch B_t of s sample indices,
//   A_t     = (1/s) sum_{i in B_t} x_i (+) x_i^T     (eq. 5 on the batch; float64 sums, stored float32)
//   w_{t+1} = A_t (+) w_t - beta w_{t-1}              (float32 product, w_{-1} = 0)
//   nu = ||w_{t+1}||_1 (float64);  w_t <- w_t / nu;  w_{t+1} <- w_{t+1} / nu
// and optionally divides w_T by its l2 norm.  The data matrix is N x D with the
// samples as rows (Algorithm 3's layout), so a gathered sample is one
// contiguous row.  D <= kMbMaxD keeps the batch matrix, a chunk of gathered
// samples and the iterates in LDS; each thread owns at most kMbPairs entries of
// the batch matrix and sums their terms in sample order.
#include "common.h"

namespace mapi {

constexpr int kMbThreads = 256;
constexpr int kMbMaxD = 64;
constexpr int kMbPairs = kMbMaxD * kMbMaxD / kMbThreads;   // 16
constexpr int kMbChunk = 128;                                // samples gathered per LDS pass

template <int OP>
__device__ __forceinline__ double mb_term(float a, float b) {
  if constexpr (OP == MAPI_OP_MIN1) {
    const float bb = fabsf(b);
    return (double)__builtin_amdgcn_fmed3f(flip_sign(a, sign_bit(b)), -bb, bb);   // exact in float32
  } else {
    return (double)a * (double)b;                                                  // exact in float64
  }
}

template <int OP>
__global__ void __launch_bounds__(kMbThreads)
k_minibatch(const float* __restrict__ X, int64_t N, int D, int64_t ldx, const int32_t* __restrict__ idx, int s, int T,
            float beta, const float* __restrict__ w0, float* __restrict__ w_out, int final_l2, MbRun* __restrict__ runs,
            int32_t* __restrict__ bad_index) {
  __shared__ float xb[kMbChunk * kMbMaxD];
  __shared__ float A[kMbMaxD * kMbMaxD];
  __shared__ float w[kMbMaxD], wp[kMbMaxD];
  __shared__ double sh[16];
  const int run = blockIdx.x, tid = threadIdx.x;
  const int DD = D * D;
  if (tid < D) {
    w[tid] = w0[(int64_t)run * D + tid];
    wp[tid] = 0.0f;
  }
  const double inv_s = 1.0 / (double)s;
  int status = MAPI_OK, it = 0;
  double nu = 0.0;
  for (int t = 0; t < T; ++t) {
    const int32_t* B = idx + ((int64_t)run * T + t) * s;
    double acc[kMbPairs];
#pragma unroll
    for (int q = 0; q < kMbPairs; ++q) acc[q] = 0.0;
    for (int i0 = 0; i0 < s; i0 += kMbChunk) {
      const int c = min(kMbChunk, s - i0);
      __syncthreads();   // the previous chunk's readers are done
      for (int e = tid; e < c * D; e += kMbThreads) {
        const int i = e / D, k = e - i * D;
        int64_t j = B[i0 + i];
        if (j < 0 || j >= N) {   // never used as an address; reported after the run
          atomicOr(bad_index, 1);
          j = 0;
        }
        xb[i * D + k] = X[j * ldx + k];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kMbPairs; ++q) {
        const int p = tid + q * kMbThreads;
        if (p < DD) {
          const int k = p / D, l = p - k * D;
          double a = acc[q];
          for (int i = 0; i < c; ++i) a += mb_term<OP>(xb[i * D + k], xb[i * D + l]);
          acc[q] = a;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kMbPairs; ++q) {
      const int p = tid + q * kMbThreads;
      if (p < DD) A[p] = (float)(acc[q] * inv_s);
    }
    __syncthreads();
    float wn = 0.0f;
    double part = 0.0;
    if (tid < D) {
      float y = 0.0f;
      for (int l = 0; l < D; ++l) y = op_acc<OP>(y, A[tid * D + l], w[l], sign_bit(w[l]));
      wn = fmaf(-beta, wp[tid], y);
      part = fabs((double)wn);
    }
    nu = block_sum_f64(part, sh);
    if (!(nu > 0.0) || !(nu < INFINITY)) {
      status = MAPI_ERR_DEGENERATE;
      break;
    }
    if (tid < D) {
      wp[tid] = (float)((double)w[tid] / nu);
      w[tid] = (float)((double)wn / nu);
    }
    ++it;
    __syncthreads();
  }
  __syncthreads();
  double scale = 1.0;
  if (final_l2 && status == MAPI_OK) {
    const double q2 = block_sum_f64(tid < D ? (double)w[tid] * (double)w[tid] : 0.0, sh);
    if (!(q2 > 0.0) || !(q2 < INFINITY)) status = MAPI_ERR_DEGENERATE;
    else scale = 1.0 / sqrt(q2);
  }
  if (tid < D) w_out[(int64_t)run * D + tid] = (scale == 1.0) ? w[tid] : (float)((double)w[tid] * scale);
  if (tid == 0) {
    runs[run].iters = it;
    runs[run].status = status;
    runs[run].nu = nu;
  }
}

int minibatch_max_d() { return kMbMaxD; }

hipError_t launch_minibatch(const float* X, int64_t N, int D, int64_t ldx, const int32_t* idx, int s, int T, float beta,
                            int op, int runs, const float* w0, float* w_out, int final_l2, MbRun* ri,
                            int32_t* bad_index, hipStream_t st) {
  if (op == MAPI_OP_MIN1)
    hipLaunchKernelGGL(k_minibatch<MAPI_OP_MIN1>, dim3(runs), dim3(kMbThreads), 0, st, X, N, D, ldx, idx, s, T, beta,
                       w0, w_out, final_l2, ri, bad_index);
  else if (op == MAPI_OP_DOT)
    hipLaunchKernelGGL(k_minibatch<MAPI_OP_DOT>, dim3(runs), dim3(kMbThreads), 0, st, X, N, D, ldx, idx, s, T, beta,
                       w0, w_out, final_l2, ri, bad_index);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace mapi
