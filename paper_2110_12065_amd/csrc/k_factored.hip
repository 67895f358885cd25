// Column products of the factored operator X (+) (X^T (+) w) -- a variant that is not a
// method of the paper: the paper forms the min-covariance (1/N) X (+) X^T first (eq. 5)
// and iterates on it, while this operator applies the two factors to w one after the
// other, streaming X twice per iteration and never forming the D x D matrix.  The row
// products X (+) z use the dense product kernel.
//
// z_k = sum_i op(X_ik, w_i) over the D rows of X (D x N, row-major, samples as columns):
// each thread owns four consecutive columns (one 16-byte load per row), a block covers
// 1024 columns, and the rows are cut into RC chunks (blockIdx.y) whose float32 partial
// sums the next kernel adds in chunk order.  Within a chunk each column is summed row by
// row, so the result depends only on (D, N, RC), never on scheduling.
#include "common.h"

namespace mapi {

constexpr int kColThreads = 256;
constexpr int kColRowsPerStep = 4;     // rows whose loads are in flight together

template <int OP>
__global__ void __launch_bounds__(kColThreads)
k_col_product(const float* __restrict__ X, int64_t D, int64_t N, int64_t ldx, const float* __restrict__ w,
              float* __restrict__ zpart, int64_t rows_per_chunk, const SolveState* __restrict__ st) {
  if (st != nullptr && state_done(st)) return;
  const int64_t c4 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < D ? r0 + rows_per_chunk : D;
  if (c4 >= N) return;
  const bool full = c4 + 3 < N;        // the last thread of a ragged row reads its valid columns only
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  auto load4 = [&](int64_t i, float* x) {
    const float* p = X + i * ldx + c4;
    if (full) {
      const float4 v = *reinterpret_cast<const float4*>(p);
      x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) x[k] = c4 + k < N ? p[k] : 0.0f;
    }
  };
  int64_t i = r0;
  for (; i + kColRowsPerStep <= r1; i += kColRowsPerStep) {
    float x[kColRowsPerStep][4];
#pragma unroll
    for (int q = 0; q < kColRowsPerStep; ++q) load4(i + q, x[q]);
#pragma unroll
    for (int q = 0; q < kColRowsPerStep; ++q) {
      const float wi = w[i + q];
      const uint32_t si = sign_bit(wi);
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] = op_acc<OP>(acc[k], x[q][k], wi, si);
    }
  }
  for (; i < r1; ++i) {
    float x[4];
    load4(i, x);
    const float wi = w[i];
    const uint32_t si = sign_bit(wi);
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = op_acc<OP>(acc[k], x[k], wi, si);
  }
  float* out = zpart + (int64_t)blockIdx.y * N + c4;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (c4 + k < N) out[k] = acc[k];
}

// z_k = sum over the RC chunks in order of the chunk partials.
__global__ void __launch_bounds__(256)
k_col_sum(const float* __restrict__ zpart, int64_t N, int RC, float* __restrict__ z, const SolveState* __restrict__ st) {
  if (st != nullptr && state_done(st)) return;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int r = 0; r < RC; ++r) s += zpart[(int64_t)r * N + k];
    z[k] = s;
  }
}

// Row chunks of the column product: about 128 rows each, at most 32, so that a wide X
// gets some thousands of blocks; a function of D only.
int col_product_chunks(int64_t D) {
  int64_t rc = D / 128;
  if (rc > 32) rc = 32;
  return (int)(rc < 1 ? 1 : rc);
}

hipError_t launch_col_product(int op, const float* X, int64_t D, int64_t N, int64_t ldx, const float* w,
                              float* zpart, float* z, const SolveState* st, hipStream_t s) {
  const int RC = col_product_chunks(D);
  const int64_t rows = (D + RC - 1) / RC;
  const dim3 grid((unsigned)((N + 4 * kColThreads - 1) / (4 * kColThreads)), (unsigned)RC);
  switch (op) {
    case MAPI_OP_MIN1:
      hipLaunchKernelGGL(k_col_product<MAPI_OP_MIN1>, grid, dim3(kColThreads), 0, s, X, D, N, ldx, w, zpart, rows, st);
      break;
    case MAPI_OP_MIN2:
      hipLaunchKernelGGL(k_col_product<MAPI_OP_MIN2>, grid, dim3(kColThreads), 0, s, X, D, N, ldx, w, zpart, rows, st);
      break;
    default: return hipErrorInvalidValue;
  }
  int64_t sb = (N + 255) / 256;
  if (sb > 4096) sb = 4096;
  hipLaunchKernelGGL(k_col_sum, dim3((unsigned)sb), dim3(256), 0, s, zpart, N, RC, z, st);
  return hipGetLastError();
}

}  // namespace mapi
