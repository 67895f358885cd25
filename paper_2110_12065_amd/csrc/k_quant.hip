// Reduced-storage conversion of a float32 matrix: bfloat16 (nearest, ties to
// even) and OCP e4m3fn with one float32 scale per row (scale = amax / 448,
// values divided by the scale, nearest, ties to even, saturating at 448).
// One-time work ahead of the iterations; bit-level encoders written from the
// format definitions.
#include "common.h"

namespace mapi {

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x0040u);   // quiet NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// e4m3fn: bias 7, 3 significand bits, largest finite 448 (0x7E), 0x7F = NaN.
__device__ __forceinline__ uint8_t e4m3fn_rne_sat(float x) {
  const uint32_t u = __float_as_uint(x);
  const uint32_t sign = (u >> 24) & 0x80u;
  const float m = fabsf(x);
  if (m != m) return (uint8_t)(sign | 0x7Fu);
  if (m >= 448.0f) return (uint8_t)(sign | 0x7Eu);
  uint32_t code;
  if (m >= 0.015625f) {                       // normal range, m >= 2^-6
    const uint32_t mu = __float_as_uint(m);
    int e = (int)(mu >> 23) - 127;            // -6 .. 8
    const uint32_t mant = mu & 0x7FFFFFu;
    const uint32_t rounded = mant + 0x7FFFFu + ((mant >> 20) & 1u);   // to 3 bits, ties to even
    uint32_t q = rounded >> 20;               // 0 .. 8
    if (q == 8u) { q = 0u; e += 1; }
    code = ((uint32_t)(e + 7) << 3) | q;      // <= 0x7E because m < 448
  } else {                                    // subnormal steps of 2^-9
    code = (uint32_t)__builtin_rintf(m * 512.0f);   // 0 .. 8; 8 is the smallest normal
  }
  return (uint8_t)(sign | code);
}

__global__ void __launch_bounds__(256)
k_quant_bf16(const float* __restrict__ A, int64_t n_rows, int64_t n_cols, int64_t lda, uint16_t* __restrict__ out,
             int64_t ldo) {
  for (int64_t i = blockIdx.x; i < n_rows; i += gridDim.x)
    for (int64_t j = threadIdx.x; j < n_cols; j += blockDim.x) out[i * ldo + j] = bf16_rne(A[i * lda + j]);
}

__global__ void __launch_bounds__(256)
k_quant_fp8_rows(const float* __restrict__ A, int64_t n_rows, int64_t n_cols, int64_t lda, uint8_t* __restrict__ out,
                 int64_t ldo, float* __restrict__ scale) {
  __shared__ float sh[4];
  for (int64_t i = blockIdx.x; i < n_rows; i += gridDim.x) {
    const float* row = A + i * lda;
    float amax = 0.0f;
    for (int64_t j = threadIdx.x; j < n_cols; j += blockDim.x) amax = fmaxf(amax, fabsf(row[j]));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off, kWave));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = amax;
    __syncthreads();
    amax = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
    // smallest power of two s = 2^k (k >= -126) with 448 s >= amax: with amax = m 2^e,
    // m in [0.5, 1), and 448 = 0.875 * 2^9, k = e - 9, plus one when m > 0.875
    int e = 0;
    const float m = frexpf(amax, &e);
    const int k = max(e - 9 + (m > 0.875f ? 1 : 0), -126);
    const float s = (amax > 0.0f) ? ldexpf(1.0f, k) : 1.0f;
    if (threadIdx.x == 0) scale[i] = s;
    for (int64_t j = threadIdx.x; j < n_cols; j += blockDim.x) out[i * ldo + j] = e4m3fn_rne_sat(__fdiv_rn(row[j], s));
  }
}

static int rows_grid(int64_t n_rows) { return (int)(n_rows < 65536 ? (n_rows < 1 ? 1 : n_rows) : 65536); }

hipError_t launch_quant_bf16(const float* A, int64_t n_rows, int64_t n_cols, int64_t lda, uint16_t* out, int64_t ldo,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_quant_bf16, dim3(rows_grid(n_rows)), dim3(256), 0, s, A, n_rows, n_cols, lda, out, ldo);
  return hipGetLastError();
}

hipError_t launch_quant_fp8(const float* A, int64_t n_rows, int64_t n_cols, int64_t lda, uint8_t* out, int64_t ldo,
                            float* scale, hipStream_t s) {
  hipLaunchKernelGGL(k_quant_fp8_rows, dim3(rows_grid(n_rows)), dim3(256), 0, s, A, n_rows, n_cols, lda, out, ldo,
                     scale);
  return hipGetLastError();
}

}  // namespace mapi
