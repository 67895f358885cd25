// PageRank products on G = alpha H + (1 - alpha)/n 1 (eq. 11) without forming G.
//
// With c = (1 - alpha)/n, every column of row i of G holds c except the
// dangling columns (1/n) and the in-links j of i (alpha H_ij + c).  For the
// min1 product (eq. 3) with G >= 0 each term is t(g, w_j) = clamp(w_j, -g, g),
// so
//   y_i = T + Dg + sum_{j in in(i)} [clamp(w_j, +-(alpha H_ij + c)) - clamp(w_j, +-c)]
//   T   = sum_j clamp(w_j, +-c),  Dg = sum_{j dangling} [clamp(w_j, +-1/n) - clamp(w_j, +-c)].
// For RPI, y_i = alpha sum_{j in in(i)} H_ij w_j + (alpha/n) sum_{dangling} w_j + c sum_j w_j.
// T, Dg (or the two sums) are float64 scalars of the current iterate, reduced by
// the normalisation kernel of the previous iteration (or k_pr_scalars for w0).
//
// Rows are destinations; G lanes of a wave share one row, stride along its
// in-links and reduce with a fixed butterfly; a lane group holds R rows at once
// to keep several gathers in flight.  In-degrees of graphs with uniformly drawn
// destinations are nearly Poisson, so short rows dominate.
#include "common.h"

namespace mapi {

__global__ void k_fill_u8(uint8_t* p, int64_t n, uint8_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Validate the CSR arrays and clear the dangling flag of every node that is a
// source.  Out-of-range entries set *err and are never used as an address.
__global__ void k_csr_check(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col, int64_t n,
                            int64_t nnz, uint8_t* __restrict__ dangling, int32_t* __restrict__ err) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (tid == 0 && (row_ptr[0] != 0 || (int64_t)row_ptr[n] != nnz)) atomicOr(err, 1);
  for (int64_t i = tid; i < n; i += stride)
    if (row_ptr[i] > row_ptr[i + 1]) atomicOr(err, 2);
  // every source in range, and a source with an out-link not dangling.  The flag is read
  // before it is cleared: most links come from sources with many links, and a read that
  // finds the flag already clear costs less than another byte write.  Each thread loads
  // U links before it touches their flags, so that the flag reads overlap.
  constexpr int U = 4;
  for (int64_t p0 = tid; p0 < nnz; p0 += stride * U) {
    int32_t j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t p = p0 + u * stride;
      j[u] = p < nnz ? col[p] : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (p0 + u * stride >= nnz) continue;
      if (j[u] < 0 || (int64_t)j[u] >= n) {
        atomicOr(err, 4);
      } else if (dangling[j[u]]) {
        dangling[j[u]] = 0;
      }
    }
  }
}

// T/Dg (MAPI) or sum/dangling-sum (RPI) of an iterate, into st->ex.
template <int METHOD, typename T>
__global__ void __launch_bounds__(256)
k_pr_scalars(const T* __restrict__ w, int64_t n, const uint8_t* __restrict__ dangling, double c, double inv_n,
             SolveState* __restrict__ st, double* __restrict__ part) {
  __shared__ double sh[16];
  __shared__ int sh_flag;
  double e0 = 0.0, e1 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double wd = (double)w[i];
    if constexpr (METHOD == MAPI_METHOD_MAPI) {
      const double tc = fmin(fmax(wd, -c), c);
      e0 += tc;
      if (dangling[i]) e1 += fmin(fmax(wd, -inv_n), inv_n) - tc;
    } else {
      e0 += wd;
      if (dangling[i]) e1 += wd;
    }
  }
  e0 = block_sum_f64(e0, sh);
  e1 = block_sum_f64(e1, sh);
  if (threadIdx.x == 0) {
    store_agent(&part[2 * (size_t)blockIdx.x], e0);
    store_agent(&part[2 * (size_t)blockIdx.x + 1], e1);
  }
  if (arrive_last(&st->cnt_b, &sh_flag)) {
    const double E0 = block_sum_parts(part, gridDim.x, 2, 0, sh);
    const double E1 = block_sum_parts(part, gridDim.x, 2, 1, sh);
    if (threadIdx.x == 0) {
      st->ex[0] = E0;
      st->ex[1] = E1;
      st->cnt_b = 0;
    }
  }
}

// G lanes per row, each summing the row's in-links k = sub, sub + G, ... in order,
// then a fixed butterfly; each lane group carries R consecutive rows at once, so a
// lane keeps R independent index / value / gather chains in flight.
// T: the iterate's type.  float: float32 terms and row sums (the clamps on v_med3_f32);
// double: every term and sum in float64 (the FP64-iterate option).
template <int METHOD, int G, int R, typename T>
__global__ void __launch_bounds__(256)
k_csr_product(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col, const float* __restrict__ val,
              int64_t n, const T* __restrict__ w, T* __restrict__ y, double* __restrict__ part,
              SolveState* __restrict__ st, double alpha, double c, double inv_n) {
  __shared__ double sh[16];
  if (state_done(st)) return;
  // the float32 iterate uses alpha and c rounded to float32 (as the batched kernel does)
  const double ad = sizeof(T) == 4 ? (double)(float)alpha : alpha;
  const double cd = sizeof(T) == 4 ? (double)(float)c : c;
  const double base = (METHOD == MAPI_METHOD_MAPI) ? st->ex[0] + st->ex[1] : (ad * inv_n) * st->ex[1] + cd * st->ex[0];
  const int sub = threadIdx.x % G;
  const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int64_t ng = ((int64_t)gridDim.x * blockDim.x) / G;
  double nrm = 0.0;
  for (int64_t i0 = gid * R; i0 < n; i0 += ng * R) {
    int32_t p0[R], len[R];
    int32_t maxlen = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool ok = i0 + r < n;
      p0[r] = ok ? row_ptr[i0 + r] : 0;
      len[r] = ok ? row_ptr[i0 + r + 1] - p0[r] : 0;
      maxlen = max(maxlen, len[r]);
    }
    const float af = (float)ad, cf = (float)cd;
    T acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = T(0);
    for (int32_t k = sub; k < maxlen; k += G) {
      int32_t cj[R];
      float h[R];
      T wj[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool ok = k < len[r];
        cj[r] = ok ? col[p0[r] + k] : 0;
        h[r] = ok ? val[p0[r] + k] : 0.0f;
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (!MAPI_DCHECK(st, (uint64_t)(uint32_t)cj[r] < (uint64_t)n, 2)) cj[r] = 0;   // a source outside 0..n-1
        wj[r] = w[cj[r]];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (k < len[r]) {
          if constexpr (METHOD == MAPI_METHOD_MAPI) {
            if constexpr (sizeof(T) == 4) {
              const float g = fmaf(af, h[r], cf);
              acc[r] += __builtin_amdgcn_fmed3f(wj[r], -g, g) - __builtin_amdgcn_fmed3f(wj[r], -cf, cf);
            } else {
              const double g = ad * (double)h[r] + cd;
              acc[r] += fmin(fmax(wj[r], -g), g) - fmin(fmax(wj[r], -cd), cd);
            }
          } else {
            acc[r] = fma((T)h[r], wj[r], acc[r]);
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      T a = acc[r];
#pragma unroll
      for (int off = G / 2; off >= 1; off >>= 1) a += __shfl_xor(a, off, G);
      if (sub == 0 && i0 + r < n) {
        const T yi = (METHOD == MAPI_METHOD_MAPI) ? (T)(base + (double)a) : (T)(ad * (double)a + base);
        y[i0 + r] = yi;
        nrm += fabs((double)yi);
      }
    }
  }
  // one partial of the normaliser per block, summed in block order by the normalisation kernel
  const double bsum = block_sum_f64(nrm, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = bsum;
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

static int grid_for(int64_t work, int per_block, int cap) {
  int64_t b = (work + per_block - 1) / per_block;
  if (b > cap) b = cap;
  return (int)(b < 1 ? 1 : b);
}

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_csr_prep(const int32_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz, uint8_t* dangling,
                           int32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, dangling, n, (uint8_t)1);
  hipLaunchKernelGGL(k_csr_check, dim3(grid_for(n > nnz ? n : nnz, 256, 8192)), dim3(256), 0, s, row_ptr, col, n,
                     nnz, dangling, err);
  return hipGetLastError();
}

int pr_scalar_blocks(int64_t n) { return grid_for(n, 1024, 1024); }

template <typename T>
hipError_t launch_pr_scalars(int method, const T* w, int64_t n, const uint8_t* dangling, double c, double inv_n,
                             SolveState* st, double* part, hipStream_t s) {
  const int b = pr_scalar_blocks(n);
  if (method == MAPI_METHOD_MAPI)
    hipLaunchKernelGGL((k_pr_scalars<MAPI_METHOD_MAPI, T>), dim3(b), dim3(256), 0, s, w, n, dangling, c, inv_n, st,
                       part);
  else
    hipLaunchKernelGGL((k_pr_scalars<MAPI_METHOD_RPI, T>), dim3(b), dim3(256), 0, s, w, n, dangling, c, inv_n, st,
                       part);
  return hipGetLastError();
}
template hipError_t launch_pr_scalars<float>(int, const float*, int64_t, const uint8_t*, double, double, SolveState*,
                                             double*, hipStream_t);
template hipError_t launch_pr_scalars<double>(int, const double*, int64_t, const uint8_t*, double, double,
                                              SolveState*, double*, hipStream_t);

constexpr int kCsrGroup = 8;   // lanes per row
constexpr int kCsrRows = 1;    // rows per lane group at once (the kernel runs at full occupancy: more rows per
                               // group only add divergence, measured 17 % slower at R = 4)

int csr_part_count(int64_t n) { return grid_for(n, 256 / kCsrGroup * kCsrRows, 4096); }

template <typename T>
hipError_t launch_csr_product(int method, const int32_t* row_ptr, const int32_t* col, const float* val, int64_t n,
                              const T* w, T* y, double* part, SolveState* st, double alpha, double c, double inv_n,
                              hipStream_t s) {
  const int b = csr_part_count(n);
  if (method == MAPI_METHOD_MAPI)
    hipLaunchKernelGGL((k_csr_product<MAPI_METHOD_MAPI, kCsrGroup, kCsrRows, T>), dim3(b), dim3(256), 0, s, row_ptr,
                       col, val, n, w, y, part, st, alpha, c, inv_n);
  else
    hipLaunchKernelGGL((k_csr_product<MAPI_METHOD_RPI, kCsrGroup, kCsrRows, T>), dim3(b), dim3(256), 0, s, row_ptr,
                       col, val, n, w, y, part, st, alpha, c, inv_n);
  return hipGetLastError();
}
template hipError_t launch_csr_product<float>(int, const int32_t*, const int32_t*, const float*, int64_t,
                                              const float*, float*, double*, SolveState*, double, double, double,
                                              hipStream_t);
template hipError_t launch_csr_product<double>(int, const int32_t*, const int32_t*, const float*, int64_t,
                                               const double*, double*, double*, SolveState*, double, double, double,
                                               hipStream_t);

}  // namespace mapi
