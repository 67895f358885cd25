// Dense product y = A (+) w (Sec. 2.1 matrix extension of eqs. 3, 4, 7; the
// ordinary product for RPI, eq. 1), with the per-iteration normaliser reduced
// in float64 (eq. 6 denominator / eq. 1 norm), plus the normalisation and
// residual kernel and the end-of-solve kernels.
//
// Layout: A row-major, rows 16-byte aligned.  Each wave owns RW rows at a time
// and its lanes stride along the columns with 16-byte loads (4 float32, 8 bf16
// or 16 e4m3 values per lane per load), so one wave load covers 1 KiB of a row.
// The RW rows share every staged w value.  w is staged once per block in LDS.
// Row sums use a fixed butterfly across the wave; block partials of the norm
// are summed in a fixed order by the block that arrives last, so results do
// not depend on timing.
#include "common.h"

namespace mapi {

template <int DT> struct Traits;
template <> struct Traits<MAPI_F32> { static constexpr int VE = 4; static constexpr int ESZ = 4; };
template <> struct Traits<MAPI_BF16> { static constexpr int VE = 8; static constexpr int ESZ = 2; };
template <> struct Traits<MAPI_FP8_E4M3> { static constexpr int VE = 16; static constexpr int ESZ = 1; };

// Decode one 16-byte vector of stored elements to float32 (FP8: times the row scale).
template <int DT>
__device__ __forceinline__ void decode_vec(const uint4 raw, float scale, float* out) {
  const uint32_t wd[4] = {raw.x, raw.y, raw.z, raw.w};
  if constexpr (DT == MAPI_F32) {
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = __uint_as_float(wd[k]);
  } else if constexpr (DT == MAPI_BF16) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      out[2 * k] = __uint_as_float(wd[k] << 16);
      out[2 * k + 1] = __uint_as_float(wd[k] & 0xFFFF0000u);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)wd[k], false);
      const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)wd[k], true);
      out[4 * k + 0] = scale * lo[0];
      out[4 * k + 1] = scale * lo[1];
      out[4 * k + 2] = scale * hi[0];
      out[4 * k + 3] = scale * hi[1];
    }
  }
}

template <int DT>
__device__ __forceinline__ float decode_one(const unsigned char* row, int64_t j, float scale) {
  if constexpr (DT == MAPI_F32) {
    return reinterpret_cast<const float*>(row)[j];
  } else if constexpr (DT == MAPI_BF16) {
    return __uint_as_float(((uint32_t)reinterpret_cast<const uint16_t*>(row)[j]) << 16);
  } else {
    return scale * __builtin_amdgcn_cvt_f32_fp8((int)row[j], 0);
  }
}

template <int DT, int OP, int RW, bool WLDS>
__global__ void __launch_bounds__(512)
k_mavp_dense(const unsigned char* __restrict__ A, int64_t ld_bytes, int n_rows, int n_cols,
             const float* __restrict__ rscale, const float* __restrict__ w, float* __restrict__ y,
             double* __restrict__ part, SolveState* __restrict__ st, int norm) {
  constexpr int VE = Traits<DT>::VE;
  constexpr int U = (DT == MAPI_F32) ? 4 : 2;   // 16-byte loads in flight per row per lane
  extern __shared__ float4 w_lds4[];
  float* w_lds = reinterpret_cast<float*>(w_lds4);
  __shared__ double sh[16];
  __shared__ int sh_flag;

  if (st != nullptr && state_done(st)) return;

  const float* wv = w;
  if constexpr (WLDS) {
    const int nv4 = n_cols >> 2;
    for (int v = threadIdx.x; v < nv4; v += blockDim.x)
      reinterpret_cast<float4*>(w_lds)[v] = reinterpret_cast<const float4*>(w)[v];
    for (int j = (nv4 << 2) + threadIdx.x; j < n_cols; j += blockDim.x) w_lds[j] = w[j];
    __syncthreads();
    wv = w_lds;
  }

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  const int ngroups = (n_rows + RW - 1) / RW;
  const int nvec = n_cols / VE;
  double nrm = 0.0;

  for (int g = blockIdx.x * nw + wave; g < ngroups; g += gridDim.x * nw) {
    const unsigned char* rp[RW];
    float sc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int row = min(g * RW + r, n_rows - 1);     // padded rows re-read the last row
      rp[r] = A + (int64_t)row * ld_bytes;
      sc[r] = (DT == MAPI_FP8_E4M3) ? rscale[row] : 1.0f;
    }
    float acc[RW][2];
#pragma unroll
    for (int r = 0; r < RW; ++r) acc[r][0] = acc[r][1] = 0.0f;

    int v = lane;
    for (; v + kWave * (U - 1) < nvec; v += kWave * U) {
      uint4 raw[U][RW];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int r = 0; r < RW; ++r)
          raw[u][r] = *reinterpret_cast<const uint4*>(rp[r] + (int64_t)(v + kWave * u) * 16);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float wf[VE];
        uint32_t ws[VE];
        const float4* wp = reinterpret_cast<const float4*>(wv + (int64_t)(v + kWave * u) * VE);
#pragma unroll
        for (int q = 0; q < VE / 4; ++q) {
          const float4 t = wp[q];
          wf[4 * q] = t.x; wf[4 * q + 1] = t.y; wf[4 * q + 2] = t.z; wf[4 * q + 3] = t.w;
        }
#pragma unroll
        for (int e = 0; e < VE; ++e) ws[e] = sign_bit(wf[e]);
#pragma unroll
        for (int r = 0; r < RW; ++r) {
          float a[VE];
          decode_vec<DT>(raw[u][r], sc[r], a);
#pragma unroll
          for (int e = 0; e < VE; ++e) acc[r][e & 1] = op_acc<OP>(acc[r][e & 1], a[e], wf[e], ws[e]);
        }
      }
    }
    for (; v < nvec; v += kWave) {
      float wf[VE];
      uint32_t ws[VE];
      const float4* wp = reinterpret_cast<const float4*>(wv + (int64_t)v * VE);
#pragma unroll
      for (int q = 0; q < VE / 4; ++q) {
        const float4 t = wp[q];
        wf[4 * q] = t.x; wf[4 * q + 1] = t.y; wf[4 * q + 2] = t.z; wf[4 * q + 3] = t.w;
      }
#pragma unroll
      for (int e = 0; e < VE; ++e) ws[e] = sign_bit(wf[e]);
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const uint4 raw = *reinterpret_cast<const uint4*>(rp[r] + (int64_t)v * 16);
        float a[VE];
        decode_vec<DT>(raw, sc[r], a);
#pragma unroll
        for (int e = 0; e < VE; ++e) acc[r][e & 1] = op_acc<OP>(acc[r][e & 1], a[e], wf[e], ws[e]);
      }
    }
    // ragged tail: fewer than VE columns past the last full vector
    const int j = nvec * VE + lane;
    if (j < n_cols) {
      const float wj = wv[j];
      const uint32_t sj = sign_bit(wj);
#pragma unroll
      for (int r = 0; r < RW; ++r) acc[r][0] = op_acc<OP>(acc[r][0], decode_one<DT>(rp[r], j, sc[r]), wj, sj);
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const float s = wave_sum_f32(acc[r][0] + acc[r][1]);
      const int row = g * RW + r;
      if (lane == 0 && row < n_rows) {
        y[row] = s;
        nrm += (norm == NORM_L2) ? (double)s * (double)s : fabs((double)s);
      }
    }
  }

  if (st == nullptr || norm == NORM_NONE) return;
  const double bsum = block_sum_f64(nrm, sh);
  if (threadIdx.x == 0) store_agent(&part[blockIdx.x], bsum);
  if (arrive_last(&st->cnt_a, &sh_flag)) {
    const double tot = block_sum_parts(part, gridDim.x, 1, 0, sh);
    if (threadIdx.x == 0) {
      st->nu = (norm == NORM_L2) ? sqrt(tot) : tot;
      st->cnt_a = 0;
    }
  }
}

// ---------------------------------------------------------------- normalise + residual
// mode 0: dense; mode 1: PageRank with the min1 product (also the clamp sums
// T and Dg of the new iterate); mode 2: PageRank RPI (sum of w, dangling sum).
template <int MODE>
__global__ void __launch_bounds__(256)
k_finalize(const float* __restrict__ y, const float* __restrict__ w_old, float* __restrict__ w_new, int64_t n,
           SolveState* __restrict__ st, double* __restrict__ part, const uint8_t* __restrict__ dangling, double c,
           double inv_n) {
  __shared__ double sh[16];
  __shared__ int sh_flag;
  if (state_done(st)) return;
  const double nu = st->nu;
  if (!(nu > 0.0) || !(nu < INFINITY)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->status = MAPI_ERR_DEGENERATE;
      st->done = 1;
    }
    return;
  }
  double r = 0.0, e0 = 0.0, e1 = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float wn = (float)((double)y[i] / nu);
    w_new[i] = wn;
    const double wd = (double)wn;
    r += fabs(wd - (double)w_old[i]);
    if constexpr (MODE == 1) {
      const double tc = fmin(fmax(wd, -c), c);
      e0 += tc;
      if (dangling[i]) e1 += fmin(fmax(wd, -inv_n), inv_n) - tc;
    } else if constexpr (MODE == 2) {
      e0 += wd;
      if (dangling[i]) e1 += wd;
    }
  }
  r = block_sum_f64(r, sh);
  if constexpr (MODE != 0) {
    e0 = block_sum_f64(e0, sh);
    e1 = block_sum_f64(e1, sh);
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
      state_advance(st, R);
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
__global__ void __launch_bounds__(1024)
k_finish(const float* __restrict__ w0buf, const float* __restrict__ w1buf, float* __restrict__ out, int64_t n,
         SolveState* __restrict__ st, int final_l2) {
  __shared__ double sh[16];
  const float* src = (st->iter & 1) ? w1buf : w0buf;
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
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) out[i] = final_l2 ? (float)((double)src[i] * scale) : src[i];
}

// ---------------------------------------------------------------- launchers
hipError_t launch_state_init(SolveState* st, int max_iters, double tol, int stall_iters, hipStream_t s) {
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, max_iters, tol, stall_iters);
  return hipGetLastError();
}

DenseTuning dense_default_tuning(const DenseArgs& a, int cu_count, int max_lds_bytes) {
  DenseTuning t;
  t.rows_per_wave = (a.n_rows >= 4096) ? 4 : (a.n_rows >= 512 ? 2 : 1);
  t.waves = 4;
  t.blocks = 0;
  t.w_in_lds = (a.n_cols * 4 + 1024 <= (int64_t)max_lds_bytes) ? 1 : 0;
  (void)cu_count;
  return t;
}

static int dense_blocks(const DenseArgs& a, const DenseTuning& t, int cu_count) {
  const int64_t groups = (a.n_rows + t.rows_per_wave - 1) / t.rows_per_wave;
  int64_t need = (groups + t.waves - 1) / t.waves;
  int64_t cap = t.blocks > 0 ? t.blocks : (int64_t)cu_count * (t.w_in_lds && a.n_cols > 8192 ? 2 : 4);
  if (need > cap) need = cap;
  return (int)(need < 1 ? 1 : need);
}

int dense_part_count(const DenseArgs& a, const DenseTuning& t, int cu_count) {
  return dense_blocks(a, t, cu_count);
}

template <int DT, int OP, int RW>
static hipError_t launch_rw(const DenseArgs& a, const float* w, float* y, double* part, SolveState* st, int norm,
                            int blocks, int waves, int w_in_lds, hipStream_t s) {
  const unsigned char* A = static_cast<const unsigned char*>(a.A);
  const int64_t ldb = a.ld * Traits<DT>::ESZ;
  if (w_in_lds) {
    hipLaunchKernelGGL((k_mavp_dense<DT, OP, RW, true>), dim3(blocks), dim3(waves * kWave),
                       (size_t)a.n_cols * sizeof(float), s, A, ldb, (int)a.n_rows, (int)a.n_cols, a.row_scale, w, y,
                       part, st, norm);
  } else {
    hipLaunchKernelGGL((k_mavp_dense<DT, OP, RW, false>), dim3(blocks), dim3(waves * kWave), 0, s, A, ldb,
                       (int)a.n_rows, (int)a.n_cols, a.row_scale, w, y, part, st, norm);
  }
  return hipGetLastError();
}

template <int DT, int OP>
static hipError_t launch_op(const DenseArgs& a, const float* w, float* y, double* part, SolveState* st, int norm,
                            const DenseTuning& t, int blocks, hipStream_t s) {
  switch (t.rows_per_wave) {
    case 1: return launch_rw<DT, OP, 1>(a, w, y, part, st, norm, blocks, t.waves, t.w_in_lds, s);
    case 2: return launch_rw<DT, OP, 2>(a, w, y, part, st, norm, blocks, t.waves, t.w_in_lds, s);
    case 4: return launch_rw<DT, OP, 4>(a, w, y, part, st, norm, blocks, t.waves, t.w_in_lds, s);
    default: return hipErrorInvalidValue;
  }
}

template <int DT>
static hipError_t launch_dt(const DenseArgs& a, int op, const float* w, float* y, double* part, SolveState* st,
                            int norm, const DenseTuning& t, int blocks, hipStream_t s) {
  switch (op) {
    case MAPI_OP_MIN1: return launch_op<DT, MAPI_OP_MIN1>(a, w, y, part, st, norm, t, blocks, s);
    case MAPI_OP_MIN2: return launch_op<DT, MAPI_OP_MIN2>(a, w, y, part, st, norm, t, blocks, s);
    case MAPI_OP_DIAMOND: return launch_op<DT, MAPI_OP_DIAMOND>(a, w, y, part, st, norm, t, blocks, s);
    case MAPI_OP_DOT: return launch_op<DT, MAPI_OP_DOT>(a, w, y, part, st, norm, t, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mavp_dense(const DenseArgs& a, int op, const float* w, float* y, double* part, SolveState* st,
                             int norm, const DenseTuning& t, int cu_count, hipStream_t s) {
  if (t.waves != 4 && t.waves != 8) return hipErrorInvalidValue;
  const int blocks = dense_blocks(a, t, cu_count);
  switch (a.dtype) {
    case MAPI_F32: return launch_dt<MAPI_F32>(a, op, w, y, part, st, norm, t, blocks, s);
    case MAPI_BF16: return launch_dt<MAPI_BF16>(a, op, w, y, part, st, norm, t, blocks, s);
    case MAPI_FP8_E4M3: return launch_dt<MAPI_FP8_E4M3>(a, op, w, y, part, st, norm, t, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

int finalize_blocks(int64_t n) {
  int64_t b = (n + 1023) / 1024;
  if (b > 1024) b = 1024;
  return (int)(b < 1 ? 1 : b);
}

hipError_t launch_finalize(int mode, const float* y, const float* w_old, float* w_new, int64_t n, SolveState* st,
                           double* part, const uint8_t* dangling, double c, double inv_n, hipStream_t s) {
  const int blocks = finalize_blocks(n);
  switch (mode) {
    case 0: hipLaunchKernelGGL(k_finalize<0>, dim3(blocks), dim3(256), 0, s, y, w_old, w_new, n, st, part, dangling, c, inv_n); break;
    case 1: hipLaunchKernelGGL(k_finalize<1>, dim3(blocks), dim3(256), 0, s, y, w_old, w_new, n, st, part, dangling, c, inv_n); break;
    case 2: hipLaunchKernelGGL(k_finalize<2>, dim3(blocks), dim3(256), 0, s, y, w_old, w_new, n, st, part, dangling, c, inv_n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finish(const float* w0buf, const float* w1buf, float* out, int64_t n, SolveState* st, int final_l2,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, w0buf, w1buf, out, n, st, final_l2);
  return hipGetLastError();
}

}  // namespace mapi
