// Image reconstruction via MAPI (Algorithm 2, Sec. 3.1): centring, the
// min-outer-product deflation C - (w1 (+) w1^T) C and the reconstruction
// (W (+) W^T)(v_i - m) + m.  The min-covariance build and the two MAPI solves use
// the Gram and dense-product kernels.
//
// Deflation without the O(P^3) product.  With a = |w1| and s = sign(w1),
// (w1 (+) w1^T)_ij = s_i s_j min(a_i, a_j) for min1 (eq. 3).  In the order of
// increasing a (ties by index), row i of rank r of the product with C is
//   s_i [ sum_{q <= r} a_(q) s_(q) C_(q),:  +  a_i sum_{q > r} s_(q) C_(q),: ],
// a prefix scan over C's rows in that order: two float64 running sums per column.
// For min2 (eq. 4) the entry is 1(s_i = s_j) min(a_i, a_j): the same scan kept
// separately over the rows of positive and of negative w1 (four running sums), and
// row i takes the pair of its own sign (a zero w1_i gives a zero row).
// The scan is split into G row segments: pass 1 sums each segment, pass 2 starts
// each segment from the sums of the segments before it (fixed order, so the result
// does not depend on scheduling).  Traffic: C read twice, C' written once.
#include "common.h"

namespace mapi {

constexpr int kImgThreads = 256;

// m_p = mean_i V[p, i] (float64 sum); Vc[p, i] = V[p, i] - m_p.
__global__ void __launch_bounds__(kImgThreads)
k_img_center(const float* __restrict__ V, int64_t P, int N, int64_t ldv, float* __restrict__ Vc, int64_t ldc,
             float* __restrict__ m) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double s = 0.0;
  for (int i = 0; i < N; ++i) s += (double)V[p * ldv + i];
  const float mp = (float)(s / (double)N);
  m[p] = mp;
  for (int i = 0; i < N; ++i) Vc[p * ldc + i] = V[p * ldv + i] - mp;
  for (int i = N; i < ldc; ++i) Vc[p * ldc + i] = 0.0f;   // pitch padding
}

// rank_i = #{j : a_j < a_i or (a_j == a_i and j < i)}, a = |w|; perm[rank_i] = i.
__global__ void __launch_bounds__(kImgThreads)
k_img_rank(const float* __restrict__ w, int64_t P, int32_t* __restrict__ perm) {
  __shared__ float sa[kImgThreads * 4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const float ai = i < P ? fabsf(w[i]) : 0.0f;
  int64_t rank = 0;
  for (int64_t j0 = 0; j0 < P; j0 += kImgThreads * 4) {
    __syncthreads();
    for (int k = threadIdx.x; k < kImgThreads * 4; k += kImgThreads)
      sa[k] = (j0 + k < P) ? fabsf(w[j0 + k]) : INFINITY;
    __syncthreads();
    const int64_t jn = (P - j0 < kImgThreads * 4) ? P - j0 : kImgThreads * 4;
    for (int64_t k = 0; k < jn; ++k) {
      const float aj = sa[k];
      rank += (aj < ai || (aj == ai && j0 + k < i)) ? 1 : 0;
    }
  }
  if (i < P) perm[rank] = (int32_t)i;
}

// Running sums per column of one scan: min1 keeps (SA, SB) = (sum a s C, sum s C); min2
// keeps (SA+, SB+, SA-, SB-) = (sum a C, sum C) over the rows of positive and of
// negative w1.
template <int OP> struct DeflSums { static constexpr int K = OP == MAPI_OP_MIN2 ? 4 : 2; };

template <int OP>
__device__ __forceinline__ void defl_add(double* acc, float wi, double x) {
  const double ai = (double)fabsf(wi);
  if constexpr (OP == MAPI_OP_MIN2) {
    if (wi > 0.0f) {
      acc[0] += ai * x;
      acc[1] += x;
    } else if (wi < 0.0f) {
      acc[2] += ai * x;
      acc[3] += x;
    }
  } else {
    const double sx = wi > 0.0f ? x : (wi < 0.0f ? -x : 0.0);
    acc[0] += ai * sx;
    acc[1] += sx;
  }
}

// Pass 1: per row segment g and column c, the segment's sums over its ranks.
template <int OP>
__global__ void __launch_bounds__(kImgThreads)
k_img_defl_sums(const float* __restrict__ C, int64_t P, int64_t ldc, const float* __restrict__ w,
                const int32_t* __restrict__ perm, int64_t seg, double* __restrict__ sums) {
  constexpr int K = DeflSums<OP>::K;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t g = blockIdx.y;
  if (c >= P) return;
  const int64_t r0 = g * seg, r1 = (r0 + seg < P) ? r0 + seg : P;
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    const int32_t i = perm[r];
    defl_add<OP>(acc, w[i], (double)C[(int64_t)i * ldc + c]);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) sums[(g * P + c) * K + k] = acc[k];
}

// Pass 2: C'_(r),c = C_(r),c - M_(r),c with, for min1, M = s_(r) (PA_r + a_(r) (TB - PB_r))
// (PA / PB the prefix sums up to and including rank r, TB the total of s C over all rows)
// and, for min2, M = PA_r + a_(r) (TB - PB_r) over the rows of w1's sign at rank r.
template <int OP>
__global__ void __launch_bounds__(kImgThreads)
k_img_defl_apply(const float* __restrict__ C, int64_t P, int64_t ldc, const float* __restrict__ w,
                 const int32_t* __restrict__ perm, int64_t seg, int G, const double* __restrict__ sums,
                 float* __restrict__ Cd) {
  constexpr int K = DeflSums<OP>::K;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t g = blockIdx.y;
  if (c >= P) return;
  double pre[K], tot[K];
#pragma unroll
  for (int k = 0; k < K; ++k) pre[k] = tot[k] = 0.0;
  for (int64_t h = 0; h < G; ++h) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double v = sums[(h * P + c) * K + k];
      if (h < g) pre[k] += v;
      tot[k] += v;
    }
  }
  const int64_t r0 = g * seg, r1 = (r0 + seg < P) ? r0 + seg : P;
  for (int64_t r = r0; r < r1; ++r) {
    const int32_t i = perm[r];
    const float wi = w[i];
    const double ai = (double)fabsf(wi);
    const double x = (double)C[(int64_t)i * ldc + c];
    defl_add<OP>(pre, wi, x);
    double d;
    if constexpr (OP == MAPI_OP_MIN2) {
      d = wi > 0.0f ? pre[0] + ai * (tot[1] - pre[1]) : (wi < 0.0f ? pre[2] + ai * (tot[3] - pre[3]) : 0.0);
    } else {
      const double mc = ai * (tot[1] - pre[1]) + pre[0];
      d = wi > 0.0f ? mc : (wi < 0.0f ? -mc : 0.0);
    }
    Cd[(int64_t)i * ldc + c] = (float)(x - d);
  }
}

// R[p, i] = sum_l M_pl Vc[l, i] + m_p with M = W (+) W^T (op of eq. 3 or 4; K = 2 columns of
// W at W and W + P) for MAPI, or M = W W^T for RPI.  One thread per pixel p, float64 sums
// over l in order; W and Vc staged through LDS.
template <int OP>
__global__ void __launch_bounds__(kImgThreads)
k_img_reconstruct(const float* __restrict__ W, const float* __restrict__ Vc, int64_t P, int N, int64_t ldc,
                  const float* __restrict__ m, float* __restrict__ R, int64_t ldr) {
  constexpr int CH = 256;
  constexpr int MAXN = 16;
  __shared__ float w1s[CH], w2s[CH];
  __shared__ float xs[CH * MAXN];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const float a1 = p < P ? W[p] : 0.0f, a2 = p < P ? W[P + p] : 0.0f;
  double acc[MAXN];
#pragma unroll
  for (int i = 0; i < MAXN; ++i) acc[i] = 0.0;
  for (int64_t l0 = 0; l0 < P; l0 += CH) {
    const int ln = (P - l0 < CH) ? (int)(P - l0) : CH;
    __syncthreads();
    for (int k = threadIdx.x; k < ln; k += kImgThreads) {
      w1s[k] = W[l0 + k];
      w2s[k] = W[P + l0 + k];
    }
    for (int k = threadIdx.x; k < ln * N; k += kImgThreads) {
      const int l = k / N, i = k - l * N;
      xs[l * MAXN + i] = Vc[(l0 + l) * ldc + i];
    }
    __syncthreads();
    if (p < P) {
      for (int l = 0; l < ln; ++l) {
        double mpl;
        if constexpr (OP == MAPI_OP_DOT) {
          mpl = (double)a1 * (double)w1s[l] + (double)a2 * (double)w2s[l];
        } else {
          mpl = (double)op_acc<OP>(0.0f, a1, w1s[l], sign_bit(w1s[l])) +
                (double)op_acc<OP>(0.0f, a2, w2s[l], sign_bit(w2s[l]));
        }
#pragma unroll
        for (int i = 0; i < MAXN; ++i)
          if (i < N) acc[i] += mpl * (double)xs[l * MAXN + i];
      }
    }
  }
  if (p < P)
    for (int i = 0; i < N; ++i) R[p * ldr + i] = (float)(acc[i] + (double)m[p]);
}

int image_max_n() { return 16; }

hipError_t launch_img_center(const float* V, int64_t P, int N, int64_t ldv, float* Vc, int64_t ldc, float* m,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_img_center, dim3((unsigned)((P + kImgThreads - 1) / kImgThreads)), dim3(kImgThreads), 0, s, V,
                     P, N, ldv, Vc, ldc, m);
  return hipGetLastError();
}

int image_defl_sums_per_column() { return 4; }

hipError_t launch_img_minouter_deflate(int op, const float* C, int64_t P, int64_t ldc, const float* w, int32_t* perm,
                                       double* sums, int G, float* Cd, hipStream_t s) {
  const unsigned cb = (unsigned)((P + kImgThreads - 1) / kImgThreads);
  const int64_t seg = (P + G - 1) / G;
  hipLaunchKernelGGL(k_img_rank, dim3(cb), dim3(kImgThreads), 0, s, w, P, perm);
  if (op == MAPI_OP_MIN1) {
    hipLaunchKernelGGL(k_img_defl_sums<MAPI_OP_MIN1>, dim3(cb, (unsigned)G), dim3(kImgThreads), 0, s, C, P, ldc, w,
                       perm, seg, sums);
    hipLaunchKernelGGL(k_img_defl_apply<MAPI_OP_MIN1>, dim3(cb, (unsigned)G), dim3(kImgThreads), 0, s, C, P, ldc, w,
                       perm, seg, G, sums, Cd);
  } else if (op == MAPI_OP_MIN2) {
    hipLaunchKernelGGL(k_img_defl_sums<MAPI_OP_MIN2>, dim3(cb, (unsigned)G), dim3(kImgThreads), 0, s, C, P, ldc, w,
                       perm, seg, sums);
    hipLaunchKernelGGL(k_img_defl_apply<MAPI_OP_MIN2>, dim3(cb, (unsigned)G), dim3(kImgThreads), 0, s, C, P, ldc, w,
                       perm, seg, G, sums, Cd);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_img_reconstruct(int op, const float* W, const float* Vc, int64_t P, int N, int64_t ldc,
                                  const float* m, float* R, int64_t ldr, hipStream_t s) {
  const unsigned b = (unsigned)((P + kImgThreads - 1) / kImgThreads);
  switch (op) {
    case MAPI_OP_MIN1: hipLaunchKernelGGL(k_img_reconstruct<MAPI_OP_MIN1>, dim3(b), dim3(kImgThreads), 0, s, W, Vc, P, N, ldc, m, R, ldr); break;
    case MAPI_OP_MIN2: hipLaunchKernelGGL(k_img_reconstruct<MAPI_OP_MIN2>, dim3(b), dim3(kImgThreads), 0, s, W, Vc, P, N, ldc, m, R, ldr); break;
    case MAPI_OP_DOT: hipLaunchKernelGGL(k_img_reconstruct<MAPI_OP_DOT>, dim3(b), dim3(kImgThreads), 0, s, W, Vc, P, N, ldc, m, R, ldr); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mapi
