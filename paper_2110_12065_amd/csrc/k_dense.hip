// Per-iteration kernels around the dense product: normalisation of the
// product by its float64 norm (eq. 6 denominator, eq. 1 norm) with the
// residual ||w_t - w_{t-1}||_1 and the stop rule, state initialisation, the
// end-of-solve copy with the optional l2 step (Algorithm 1), and the dispatch
// of the product kernel (dense_kernel.h) by storage type.
#include "common.h"

namespace mapi {

// ---------------------------------------------------------------- normalise + residual
// mode 0: dense; mode 1: PageRank with the min1 product (also the clamp sums
// T and Dg of the new iterate); mode 2: PageRank RPI (sum of w, dangling sum).
// Every block first sums the product kernel's per-block partials pprod[0..nprod)
// in block order (the same float64 value in every block), so the product kernel
// needs no grid-wide arrival; norm NORM_L2 takes the square root (RPI, eq. 1).
template <int MODE, int BS, int PF, typename T = float>
__global__ void __launch_bounds__(BS)
k_finalize(const T* __restrict__ y, const T* __restrict__ w_old, T* __restrict__ w_new, int64_t n,
           SolveState* __restrict__ st, const double* __restrict__ pprod, int nprod, int norm,
           double* __restrict__ part, const uint8_t* __restrict__ dangling, double c, double inv_n,
           const double* __restrict__ rprev, int nrprev) {
  __shared__ double sh[16];
  __shared__ int sh_flag;
  // The state, the first PF elements' y and w_old and the partials are all loaded before
  // any of them is used, so the prologue waits for one memory round trip; a solve that
  // is already done returns after these (harmless) loads.
  const bool done0 = state_done(st);
  const double tol = st->tol;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  StopSnap snap{};
  if (lead) snap = stop_snap(st);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  T yp[PF], wp[PF];
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    const int64_t i = i0 + k * stride;
    yp[k] = i < n ? y[i] : T(0);
    wp[k] = i < n ? w_old[i] : T(0);
  }
  const double r0 = rprev != nullptr ? wave_sum_parts(rprev, nrprev) : 0.0;
  const double tot = wave_sum_parts(pprod, nprod);
  if (done0) return;
  bool stopped = false;
  if (rprev != nullptr) {
    // the previous iteration's residual (its iterate was formed inside a product):
    // the same fixed-order sum and tolerance decision in every block; block 0
    // advances the stop rule for it
    if (lead) stopped = state_advance_from(st, snap, r0);
    if (r0 < tol) return;
  }
  const double nu = (norm == NORM_L2) ? sqrt(tot) : tot;
  // block 0's thread 0 alone writes the state; it skips this iteration if it has just
  // stopped the solve on the stall rule
  const bool owner = lead && !stopped;
  if (owner) st->nu = nu;
  if (!(nu > 0.0) || !(nu < INFINITY)) {
    if (owner) {
      st->status = MAPI_ERR_DEGENERATE;
      st->done = 1;
    }
    return;
  }
  // w = y * (1 / nu): the same arithmetic as a product that forms w itself (FusedPrev)
  const double inv = 1.0 / nu;
  double r = 0.0, e0 = 0.0, e1 = 0.0;
  auto element = [&](int64_t i, T yi, T wo) {
    const T wn = (T)((double)yi * inv);
    w_new[i] = wn;
    const double wd = (double)wn;
    r += fabs(wd - (double)wo);
    if constexpr (MODE == 1) {
      const double tc = fmin(fmax(wd, -c), c);
      e0 += tc;
      if (dangling[i]) e1 += fmin(fmax(wd, -inv_n), inv_n) - tc;
    } else if constexpr (MODE == 2) {
      e0 += wd;
      if (dangling[i]) e1 += wd;
    }
  };
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    const int64_t i = i0 + k * stride;
    if (i < n) element(i, yp[k], wp[k]);
  }
  for (int64_t i = i0 + PF * stride; i < n; i += stride) element(i, y[i], w_old[i]);
  r = block_sum_f64(r, sh);
  if constexpr (MODE != 0) {
    e0 = block_sum_f64(e0, sh);
    e1 = block_sum_f64(e1, sh);
  }
  // (a stall stop of the previous iteration, taken by block 0 above, leaves the state
  // done: this iteration is then not counted)
  if (gridDim.x == 1) {   // one block holds every sum: no partials, no arrival
    if (threadIdx.x == 0) {
      st->ex[0] = e0;
      st->ex[1] = e1;
      if (!state_done(st)) state_advance(st, r);
    }
    return;
  }
  if (threadIdx.x == 0) {
    store_agent(&part[3 * (size_t)blockIdx.x + 0], r);
    store_agent(&part[3 * (size_t)blockIdx.x + 1], e0);
    store_agent(&part[3 * (size_t)blockIdx.x + 2], e1);
  }
  if (arrive_last(&st->cnt_b, &sh_flag)) {
    const double R = block_sum_parts(part, gridDim.x, 3, 0, sh);
    double E0 = 0.0, E1 = 0.0;
    if constexpr (MODE != 0) {
      E0 = block_sum_parts(part, gridDim.x, 3, 1, sh);
      E1 = block_sum_parts(part, gridDim.x, 3, 2, sh);
    }
    if (threadIdx.x == 0) {
      st->ex[0] = E0;
      st->ex[1] = E1;
      st->cnt_b = 0;
      if (!state_done(st)) state_advance(st, R);
    }
  }
}

__global__ void k_state_init(SolveState* st, int max_iters, double tol, int stall_iters) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    SolveState s{};
    s.best_r = INFINITY;
    s.tol = tol;
    s.max_iters = max_iters;
    s.stall_iters = stall_iters;
    s.done = (max_iters <= 0) ? 1 : 0;
    *st = s;
  }
}

// Copy the final iterate (buffer chosen by the parity of the completed
// iteration count) to `out`, optionally divided by its l2 norm (Algorithm 1,
// last step).  One block; the norm is a fixed-order float64 sum.
template <typename T>
__global__ void __launch_bounds__(1024)
k_finish(const T* __restrict__ w0buf, const T* __restrict__ w1buf, T* __restrict__ out, int64_t n,
         SolveState* __restrict__ st, int final_l2) {
  __shared__ double sh[16];
  const T* src = (st->iter & 1) ? w1buf : w0buf;
  double scale = 1.0;
  if (final_l2) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += (double)src[i] * (double)src[i];
    s = block_sum_f64(s, sh);
    if (!(s > 0.0) || !(s < INFINITY)) {
      if (threadIdx.x == 0) st->status = MAPI_ERR_DEGENERATE;
      return;
    }
    scale = 1.0 / sqrt(s);
  }
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) out[i] = final_l2 ? (T)((double)src[i] * scale) : src[i];
}

// The same for long vectors (more than kFinishOneBlock elements), over many blocks: the
// squares summed per block into part[], then every block sums those in block order (the
// same bits in each) and scales or copies its share.
constexpr int64_t kFinishOneBlock = 65536;
static int finish_blocks(int64_t n) {
  const int64_t b = (n + 4095) / 4096;
  return (int)(b > 256 ? 256 : (b < 1 ? 1 : b));
}

template <typename T>
__global__ void __launch_bounds__(256)
k_finish_sq(const T* __restrict__ w0buf, const T* __restrict__ w1buf, int64_t n, const SolveState* __restrict__ st,
            double* __restrict__ part) {
  __shared__ double sh[16];
  const T* src = (st->iter & 1) ? w1buf : w0buf;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += (double)src[i] * (double)src[i];
  s = block_sum_f64(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_finish_out(const T* __restrict__ w0buf, const T* __restrict__ w1buf, T* __restrict__ out, int64_t n,
             SolveState* __restrict__ st, int final_l2, const double* __restrict__ part, int nparts) {
  const T* src = (st->iter & 1) ? w1buf : w0buf;
  double scale = 1.0;
  if (final_l2) {
    const double s = wave_sum_parts(part, nparts);
    if (!(s > 0.0) || !(s < INFINITY)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) st->status = MAPI_ERR_DEGENERATE;
      return;
    }
    scale = 1.0 / sqrt(s);
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = final_l2 ? (T)((double)src[i] * scale) : src[i];
}

// A check that always fails (device-checked builds, when the context was created with
// MAPI_DCHECK_SELFTEST=1): exercises the path from a failed device check to the caller's
// error without any out-of-bounds access.
__global__ void k_dcheck_selftest(SolveState* st) {
  if (threadIdx.x == 0) (void)MAPI_DCHECK(st, false, 15);
}

hipError_t launch_dcheck_selftest(SolveState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_dcheck_selftest, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------- launchers
hipError_t launch_state_init(SolveState* st, int max_iters, double tol, int stall_iters, hipStream_t s) {
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, max_iters, tol, stall_iters);
  return hipGetLastError();
}

DenseTuning dense_default_tuning(const DenseArgs& a, int cu_count, int max_lds_bytes) {
  // Starting shapes from a sweep at n = 16384 on MI355X (the autotuner refines
  // them per size bucket): the matrix is streamed once per product, so
  // non-temporal loads and 8 waves per block keep the most bytes in flight.
  DenseTuning t;
  const bool lds_fits = (int64_t)dense_lds_bytes(a.dtype, a.n_cols, 1) + 1024 <= (int64_t)max_lds_bytes;
  t.blocks = 0;
  t.waves = 8;
  // non-temporal loads only for a matrix larger than the 256 MB Infinity Cache: a smaller
  // one (the PCA's 4096 x 4096 matrices, 64 MiB) can stay there between products
  const int64_t bytes = a.n_rows * a.n_cols * (a.dtype == MAPI_F32 ? 4 : a.dtype == MAPI_BF16 ? 2 : 1);
  t.nontemporal = bytes > (int64_t(192) << 20) ? 1 : 0;
  if (a.dtype == MAPI_F32) {
    // enough row groups for every compute unit's 8 waves twice over (4096 rows: one row
    // per wave, two blocks per compute unit)
    const int64_t per = 2 * (int64_t)cu_count * 8;
    t.rows_per_wave = (a.n_rows >= 4 * per) ? 4 : (a.n_rows >= 2 * per ? 2 : 1);
    t.unroll = 2;
    t.blocks_per_cu = a.n_rows >= 4 * per ? 1 : 2;
    // staged w lets a solve form each iterate inside the next product (no normalisation
    // launch per iteration)
    t.w_in_lds = lds_fits ? 1 : 0;
  } else {
    t.rows_per_wave = 1;
    t.unroll = (a.dtype == MAPI_BF16) ? 4 : 2;
    t.waves = (a.dtype == MAPI_BF16) ? 4 : 8;
    t.blocks_per_cu = 2;
    t.w_in_lds = lds_fits ? 1 : 0;
  }
  return t;
}

static int dense_blocks(const DenseArgs& a, const DenseTuning& t, int cu_count) {
  const int64_t groups = (a.n_rows + t.rows_per_wave - 1) / t.rows_per_wave;
  int64_t need = (groups + t.waves - 1) / t.waves;
  const int per_cu = t.blocks_per_cu > 0 ? t.blocks_per_cu : (t.w_in_lds && a.n_cols > 8192 ? 2 : 4);
  int64_t cap = t.blocks > 0 ? t.blocks : (int64_t)cu_count * per_cu;
  if (need > cap) need = cap;
  return (int)(need < 1 ? 1 : need);
}

int dense_part_count(const DenseArgs& a, const DenseTuning& t, int cu_count) {
  return dense_blocks(a, t, cu_count);
}

hipError_t launch_dense_f32(const DenseArgs& a, int op, const float* w, float* y, double* part, SolveState* st,
                            int norm, const DenseTuning& t, int blocks, hipStream_t s, const FusedPrev* fp);
hipError_t launch_dense_bf16(const DenseArgs& a, int op, const float* w, float* y, double* part, SolveState* st,
                             int norm, const DenseTuning& t, int blocks, hipStream_t s, const FusedPrev* fp);
hipError_t launch_dense_fp8(const DenseArgs& a, int op, const float* w, float* y, double* part, SolveState* st,
                            int norm, const DenseTuning& t, int blocks, hipStream_t s, const FusedPrev* fp);

hipError_t launch_mavp_dense(const DenseArgs& a, int op, const float* w, float* y, double* part, SolveState* st,
                             int norm, const DenseTuning& t, int cu_count, hipStream_t s, const FusedPrev* fp) {
  if (t.waves != 4 && t.waves != 8) return hipErrorInvalidValue;
  const int blocks = dense_blocks(a, t, cu_count);
  switch (a.dtype) {
    case MAPI_F32: return launch_dense_f32(a, op, w, y, part, st, norm, t, blocks, s, fp);
    case MAPI_BF16: return launch_dense_bf16(a, op, w, y, part, st, norm, t, blocks, s, fp);
    case MAPI_FP8_E4M3: return launch_dense_fp8(a, op, w, y, part, st, norm, t, blocks, s, fp);
    default: return hipErrorInvalidValue;
  }
}

// Plain 16-byte copy: the bandwidth and counter reference for the product kernels.
__global__ void __launch_bounds__(256) k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

hipError_t launch_copy16(const void* src, void* dst, int64_t n16, int cu_count, hipStream_t s) {
  int64_t blocks = (n16 + 255) / 256;
  if (blocks > (int64_t)cu_count * 16) blocks = (int64_t)cu_count * 16;
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)(blocks < 1 ? 1 : blocks)), dim3(256), 0, s,
                     static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
  return hipGetLastError();
}

typedef unsigned int vec_u32x4 __attribute__((ext_vector_type(4)));

// Plain streaming read (16-byte non-temporal loads, U per lane in flight): the
// attainable-read-bandwidth reference for the product kernels.  The loaded words
// are folded into one value that is stored only if it equals a constant no input
// here produces, so the loads stay but nothing is written.
template <int U>
__global__ void __launch_bounds__(256) k_read16(const vec_u32x4* __restrict__ src, int64_t n16, uint32_t* sink) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0u;
  for (; i + (U - 1) * stride < n16; i += U * stride) {
    vec_u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < U; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (; i < n16; i += stride) {
    const vec_u32x4 v = __builtin_nontemporal_load(src + i);
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == 0x9E3779B9u) sink[0] = acc;
}

hipError_t launch_read16(const void* src, int64_t n16, uint32_t* sink, int blocks, int unroll, hipStream_t s) {
  int64_t b = (n16 + 255) / 256;
  if (b > blocks) b = blocks;
  const dim3 grid((unsigned)(b < 1 ? 1 : b));
  const auto* p = static_cast<const vec_u32x4*>(src);
  if (unroll == 8) hipLaunchKernelGGL(k_read16<8>, grid, dim3(256), 0, s, p, n16, sink);
  else if (unroll == 4) hipLaunchKernelGGL(k_read16<4>, grid, dim3(256), 0, s, p, n16, sink);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// At most one normalisation block per compute unit: the blocks' arrivals on one
// counter are serialised, so fewer, longer blocks finish sooner for large n.  (One
// block of 1024 threads for n <= 64K, which needs no arrival, measured slower: it
// cannot start until a whole compute unit is free of the product's last blocks.)
int finalize_blocks(int64_t n) {
  int64_t b = (n + 1023) / 1024;
  if (b > 256) b = 256;
  return (int)(b < 1 ? 1 : b);
}

hipError_t launch_finalize(int mode, const float* y, const float* w_old, float* w_new, int64_t n, SolveState* st,
                           const double* pprod, int nprod, int norm, double* part, const uint8_t* dangling, double c,
                           double inv_n, hipStream_t s, const double* rprev, int nrprev) {
  const int blocks = finalize_blocks(n);
  if (mode != 0 && rprev != nullptr) return hipErrorInvalidValue;
  switch (mode) {
    case 0: hipLaunchKernelGGL((k_finalize<0, 256, 4>), dim3(blocks), dim3(256), 0, s, y, w_old, w_new, n, st, pprod, nprod, norm, part, dangling, c, inv_n, rprev, nrprev); break;
    case 1: hipLaunchKernelGGL((k_finalize<1, 256, 4>), dim3(blocks), dim3(256), 0, s, y, w_old, w_new, n, st, pprod, nprod, norm, part, dangling, c, inv_n, rprev, nrprev); break;
    case 2: hipLaunchKernelGGL((k_finalize<2, 256, 4>), dim3(blocks), dim3(256), 0, s, y, w_old, w_new, n, st, pprod, nprod, norm, part, dangling, c, inv_n, rprev, nrprev); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t finish_any(const T* w0buf, const T* w1buf, T* out, int64_t n, SolveState* st, int final_l2,
                             double* part, hipStream_t s) {
  if (n <= kFinishOneBlock || part == nullptr) {
    hipLaunchKernelGGL(k_finish<T>, dim3(1), dim3(1024), 0, s, w0buf, w1buf, out, n, st, final_l2);
  } else {
    const int b = finish_blocks(n);
    if (final_l2) hipLaunchKernelGGL(k_finish_sq<T>, dim3(b), dim3(256), 0, s, w0buf, w1buf, n, st, part);
    hipLaunchKernelGGL(k_finish_out<T>, dim3(b), dim3(256), 0, s, w0buf, w1buf, out, n, st, final_l2, part, b);
  }
  return hipGetLastError();
}

hipError_t launch_finish(const float* w0buf, const float* w1buf, float* out, int64_t n, SolveState* st, int final_l2,
                         hipStream_t s, double* part) {
  return finish_any<float>(w0buf, w1buf, out, n, st, final_l2, part, s);
}

hipError_t launch_finish_f64(const double* w0buf, const double* w1buf, double* out, int64_t n, SolveState* st,
                             int final_l2, hipStream_t s, double* part) {
  return finish_any<double>(w0buf, w1buf, out, n, st, final_l2, part, s);
}

hipError_t launch_finalize_f64(int mode, const double* y, const double* w_old, double* w_new, int64_t n,
                               SolveState* st, const double* pprod, int nprod, double* part, const uint8_t* dangling,
                               double c, double inv_n, hipStream_t s) {
  const int blocks = finalize_blocks(n);
  switch (mode) {
    case 1: hipLaunchKernelGGL((k_finalize<1, 256, 4, double>), dim3(blocks), dim3(256), 0, s, y, w_old, w_new, n, st, pprod, nprod, NORM_L1, part, dangling, c, inv_n, nullptr, 0); break;
    case 2: hipLaunchKernelGGL((k_finalize<2, 256, 4, double>), dim3(blocks), dim3(256), 0, s, y, w_old, w_new, n, st, pprod, nprod, NORM_L1, part, dangling, c, inv_n, nullptr, 0); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mapi
