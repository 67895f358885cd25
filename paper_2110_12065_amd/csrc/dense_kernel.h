// Dense product kernel y = A (+) w (Sec. 2.1 matrix extension of eqs. 3, 4, 7;
// the ordinary product for RPI, eq. 1), templated on storage type, product,
// rows per wave, loads in flight, LDS staging of w and non-temporal loads.
// Included by one translation unit per storage type.
//
// Layout: A row-major, rows 16-byte aligned.  Each wave owns RW rows at a time
// and its lanes stride along the columns with 16-byte loads (4 float32, 8 bf16
// or 16 e4m3 values per lane per load), so one wave load covers 1 KiB of a row.
// The RW rows share every staged w value and its sign.  Row sums use a fixed
// butterfly across the wave; the block partials of the norm are summed in a
// fixed order by the next kernel, so results do not depend on timing.
#pragma once
#include <hip/hip_ext.h>

#include "common.h"

namespace mapi {

template <int DT> struct Traits;
template <> struct Traits<MAPI_F32> { static constexpr int VE = 4; static constexpr int ESZ = 4; };
template <> struct Traits<MAPI_BF16> { static constexpr int VE = 8; static constexpr int ESZ = 2; };
template <> struct Traits<MAPI_FP8_E4M3> { static constexpr int VE = 16; static constexpr int ESZ = 1; };

// Chunk-interleaved LDS order of w: 16-byte matrix vectors in groups of 64 (one
// per lane of a wave); within a group, chunk q (the q-th float4 of the vector's
// VE weights) of the group's l-th vector sits at float4 q * 64 + l.  A wave
// reading chunk q of 64 consecutive vectors touches one contiguous 1 KiB, and
// chunk q is a fixed offset from chunk 0.  For float32 the order is the natural
// one.  Columns past the last whole vector are not staged.
template <int DT>
__device__ __forceinline__ int perm_base(int v) {
  constexpr int Q = Traits<DT>::VE / 4;
  return (v & ~63) * Q + (v & 63);
}

// Decode one 16-byte vector of stored elements to float32 (FP8: times the row scale).
// P2 (FP8 rows whose scale is a positive power of two): the gfx950 scaled conversion
// applies the scale's exponent inside the conversion, which for such scales is the
// exact product, one instruction per two values instead of a conversion and two
// multiplies.
__device__ __forceinline__ bool pow2_scale(float s) {
  const uint32_t u = __float_as_uint(s);
  const uint32_t ex = (u >> 23) & 0xFFu;
  return (u & 0x807FFFFFu) == 0u && ex != 0u && ex != 0xFFu;
}

template <int DT, bool P2 = false>
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
  } else if constexpr (P2) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const auto lo = __builtin_amdgcn_cvt_scalef32_pk_f32_fp8((int)wd[k], scale, false);
      const auto hi = __builtin_amdgcn_cvt_scalef32_pk_f32_fp8((int)wd[k], scale, true);
      out[4 * k + 0] = lo[0];
      out[4 * k + 1] = lo[1];
      out[4 * k + 2] = hi[0];
      out[4 * k + 3] = hi[1];
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

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Reads of w staged in LDS through pointers in the LDS address space: through a generic
// pointer the compiler may emit flat loads, which count against the vector-memory
// counter, so waiting for w also waits for every matrix load in flight.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) const f32x4 lds_f32x4;
typedef __attribute__((address_space(3))) const u32x4 lds_u32x4;

typedef __attribute__((address_space(1))) const u32x4 gmem_u32x4;
typedef __attribute__((address_space(1))) const f32x4 gmem_f32x4;

// One 16-byte load of the matrix (device memory, read as such: a pointer taken from an
// instance descriptor would otherwise give a flat load); NT marks it non-temporal
// (streamed once).
template <bool NT>
__device__ __forceinline__ uint4 load16(const unsigned char* p) {
  const gmem_u32x4* gp = (const gmem_u32x4*)p;
  u32x4 v;
  if constexpr (NT) {
    v = __builtin_nontemporal_load(gp);
  } else {
    v = *gp;
  }
  return make_uint4(v.x, v.y, v.z, v.w);
}

// First wave-step of a row's visit order (see rows_product): the same for the 8 rows of
// every aligned block of 8, so that a row's sum does not depend on how many rows a wave
// takes at once (1, 2, 4 or 8, groups aligned to that count).
__device__ __forceinline__ int rot_step(int row0, int S) {
  return S > 1 ? (int)(((uint32_t)(row0 >> 3) * 7u) % (uint32_t)S) : 0;
}

// Row products of RW rows (byte pointers rp, FP8 row scales sc) against w (wv,
// n_cols floats, 16-byte aligned) by one wave: lanes stride along the columns in
// 16-byte vectors, then a fixed butterfly; out[r] is valid in every lane.
//
// PF (FP8 with w_in_lds mode 2): wv holds |w| and smask one word per 4 stored
// values whose bits 7, 15, 23, 31 are the signs of those columns' w.  One xor
// flips the signs of four stored values before decoding, so each term is
// op(a * sign(w), |w|) -- the same value as op(a, w) -- without per-element sign
// work.  wsign: the signed w, used for the ragged tail.
//
// PERM: wv is in LDS in chunk-interleaved order (perm_base), so each 16-byte LDS
// read of a wave covers one contiguous 1 KiB instead of a lane stride of VE * 4
// bytes, which puts 2 (bf16) or 4 (FP8) lanes of every 8 on the same banks; the
// ragged tail then reads wsign (w in global memory).
// WSP: address space of w when it is not in chunk-interleaved LDS order: 1 device
// memory, 3 LDS, 0 either (generic reads).
//
// Order: the row's S = nvec / 64 whole wave-steps (64 consecutive 16-byte vectors, one per
// lane) are visited from step s0 on, wrapping around, then the partial last step, then the
// ragged tail; each lane adds its terms in that order, whatever U.  s0 = rot_step(first
// row, S) staggers where concurrent waves read: with every wave starting at column 0, the
// rows' streams stay in step and a plain row-wise read measured 5-8 % slower than with
// staggered starts.
//
// first, use_first: the loads of the lane's first U wave-steps, issued earlier by the
// caller (when the row has at least U of them), used in place of loading them again.
template <int DT, int OP, int RW, int U, bool NT, bool PF = false, bool P2 = false, bool PERM = false, int WSP = 0>
__device__ __forceinline__ void rows_product(const unsigned char* const* rp, const float* sc, const float* wv,
                                             int n_cols, int lane, float* out, const uint32_t* smask,
                                             const float* wsign, const uint4 (&first)[U][RW], bool use_first,
                                             int s0) {
  constexpr int VE = Traits<DT>::VE;
  const int nvec = n_cols / VE;
  float acc[RW][2];
#pragma unroll
  for (int r = 0; r < RW; ++r) acc[r][0] = acc[r][1] = 0.0f;

  // terms of one 16-byte vector index vv for every row
  auto vec = [&](int vv, const uint4* raws) {
    float wf[VE];
    uint32_t ws[VE];
#pragma unroll
    for (int q = 0; q < VE / 4; ++q) {
      f32x4 t;
      if constexpr (PERM)
        t = ((lds_f32x4*)(wv + 4 * (int64_t)perm_base<DT>(vv)))[q * 64];
      else if constexpr (WSP == 3)
        t = ((lds_f32x4*)(wv + (int64_t)vv * VE))[q];
      else if constexpr (WSP == 1)
        t = ((gmem_f32x4*)(wv + (int64_t)vv * VE))[q];
      else
        t = reinterpret_cast<const f32x4*>(wv + (int64_t)vv * VE)[q];
      wf[4 * q] = t.x; wf[4 * q + 1] = t.y; wf[4 * q + 2] = t.z; wf[4 * q + 3] = t.w;
    }
    uint4 m = make_uint4(0u, 0u, 0u, 0u);
    if constexpr (PF) {
      const u32x4 mv = *((lds_u32x4*)(smask + (int64_t)vv * 4));
      m = make_uint4(mv.x, mv.y, mv.z, mv.w);
#pragma unroll
      for (int e = 0; e < VE; ++e) ws[e] = 0u;
    } else {
#pragma unroll
      for (int e = 0; e < VE; ++e) ws[e] = sign_bit(wf[e]);
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      uint4 rr = raws[r];
      if constexpr (PF) {
        rr.x ^= m.x; rr.y ^= m.y; rr.z ^= m.z; rr.w ^= m.w;
      }
      float a[VE];
      decode_vec<DT, P2>(rr, sc[r], a);
#pragma unroll
      for (int e = 0; e < VE; ++e) acc[r][e & 1] = op_acc<OP>(acc[r][e & 1], a[e], wf[e], ws[e]);
    }
  };

  const int S = nvec / kWave;
  // vector of this lane at visit j (j < S): wave-step (s0 + j) mod S
  auto step_v = [&](int j) {
    int st = s0 + j;
    if (st >= S) st -= S;
    return st * kWave + lane;
  };
  int j = 0;
  if (use_first && U <= S) {
#pragma unroll
    for (int u = 0; u < U; ++u) vec(step_v(u), first[u]);
    j = U;
  }
  for (; j + U <= S; j += U) {
    uint4 raw[U][RW];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int r = 0; r < RW; ++r)
        raw[u][r] = load16<NT>(rp[r] + (int64_t)step_v(j + u) * 16);
#pragma unroll
    for (int u = 0; u < U; ++u) vec(step_v(j + u), raw[u]);
  }
  for (; j < S; ++j) {
    const int v = step_v(j);
    uint4 raw[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) raw[r] = load16<NT>(rp[r] + (int64_t)v * 16);
    vec(v, raw);
  }
  if (S * kWave + lane < nvec) {   // the partial last wave-step
    const int v = S * kWave + lane;
    uint4 raw[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) raw[r] = load16<NT>(rp[r] + (int64_t)v * 16);
    vec(v, raw);
  }
  // ragged tail: fewer than VE columns past the last full vector
  const int jt = nvec * VE + lane;
  if (jt < n_cols) {
    const float wj = (PF || PERM) ? wsign[jt] : wv[jt];
    const uint32_t sj = sign_bit(wj);
#pragma unroll
    for (int r = 0; r < RW; ++r) acc[r][0] = op_acc<OP>(acc[r][0], decode_one<DT>(rp[r], jt, sc[r]), wj, sj);
  }
#pragma unroll
  for (int r = 0; r < RW; ++r) out[r] = wave_sum_f32(acc[r][0] + acc[r][1]);
}

template <int DT, int OP, int RW, int U, int WL, bool NT>
__global__ void __launch_bounds__(512)
k_mavp_dense(const unsigned char* __restrict__ A, int64_t ld_bytes, int n_rows, int n_cols,
             const float* __restrict__ rscale, const float* __restrict__ w, float* __restrict__ y,
             double* __restrict__ part, SolveState* __restrict__ st, int norm, FusedPrev fp, int rev) {
  extern __shared__ float4 w_lds4[];
  float* w_lds = reinterpret_cast<float*>(w_lds4);
  __shared__ double sh[16];

  // a product that forms its iterate checks the state after its first loads (below)
  if (!(WL != 0 && fp.y_prev != nullptr) && st != nullptr && state_done(st)) return;

  constexpr bool PF = WL == 2 && DT == MAPI_FP8_E4M3;
  constexpr bool WLDS = WL != 0;
  constexpr int VE = Traits<DT>::VE;
  const int nvec = n_cols / VE;
  const float* wv = w;
  const float* wtail = w;   // signed w of the columns past the last whole vector
  const uint32_t* smask = nullptr;
  double racc = 0.0;        // FusedPrev: this thread's part of ||w_t - w_{t-1}||_1
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  const int ngroups = (n_rows + RW - 1) / RW;
  // The loads of the wave's first row group's first step need nothing the prologue
  // forms: with w staged in LDS they are issued right after the prologue's own loads,
  // so the matrix stream starts while the prologue waits and computes.
  // (the heavier shapes keep their registers for the loop: there the loads issued ahead
  // make the compiler spill)
  constexpr bool kAhead = DT == MAPI_F32 ? RW * U <= (OP == MAPI_OP_DIAMOND ? 8 : 16)
                                         : (RW * U <= 8 && (DT == MAPI_BF16 || RW <= 2));
  uint4 first[U][RW];
  bool have_first = false;
  const int S = nvec / kWave;
  auto issue_first = [&]() {
    const int g0 = blockIdx.x * nw + wave;
    if (kAhead && g0 < ngroups && U <= S) {
      const int g = rev ? ngroups - 1 - g0 : g0;
      const int s0 = rot_step(g * RW, S);
      const unsigned char* fp0[RW];
#pragma unroll
      for (int r = 0; r < RW; ++r) fp0[r] = A + (int64_t)min(g * RW + r, n_rows - 1) * ld_bytes;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        int stp = s0 + u;
        if (stp >= S) stp -= S;
#pragma unroll
        for (int r = 0; r < RW; ++r) first[u][r] = load16<NT>(fp0[r] + (int64_t)(stp * kWave + lane) * 16);
      }
      have_first = true;
    }
  };
  if constexpr (WLDS) {
    // FusedPrev: w = y_prev * (1 / nu), nu from the previous product's partials (the
    // normalisation kernel's arithmetic); this block also writes its share of w and
    // the residual partial of that share.
    const bool fused = fp.y_prev != nullptr;
    constexpr int PQ = 8;   // float4s of y_prev per thread loaded before nu is known
    const int np4 = nvec * (VE / 4);
    const float4* src = reinterpret_cast<const float4*>(fused ? fp.y_prev : w);
    float4 pre[PQ];
    // this block's share of the new iterate: elements e0 .. e1-1, the first blockDim
    // of them also loaded before nu is known
    const int64_t per = ((int64_t)n_cols + gridDim.x - 1) / gridDim.x;
    const int64_t e0 = (int64_t)blockIdx.x * per, e1 = min((int64_t)n_cols, e0 + per);
    float ys = 0.0f, wo = 0.0f;
    // The state, the previous launch's partials and the first part of y_prev are all
    // loaded before any of them is used, so the prologue waits for one memory round
    // trip; a solve that is already done returns after these (harmless) loads.
    bool done0 = false;
    double tol = 0.0;
    StopSnap snap{};
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (fused) {
      done0 = state_done(st);
      tol = st->tol;
      if (lead) snap = stop_snap(st);
#pragma unroll
      for (int q = 0; q < PQ; ++q) {
        const int k = threadIdx.x + q * blockDim.x;
        pre[q] = k < np4 ? src[k] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
      if (e0 + threadIdx.x < e1) {
        ys = fp.y_prev[e0 + threadIdx.x];
        wo = fp.w_old[e0 + threadIdx.x];
      }
    }
    double inv = 0.0;
    if (fused) {
      double pr[kPartsPre], pt[kPartsPre];
      if (fp.rpart_prev != nullptr) parts_load(fp.rpart_prev, fp.nparts, pr);
      parts_load(fp.part_prev, fp.nparts, pt);
      issue_first();
      const double rprev = fp.rpart_prev != nullptr ? parts_sum(fp.rpart_prev, fp.nparts, pr) : 0.0;
      const double tot = parts_sum(fp.part_prev, fp.nparts, pt);
      if (done0) return;
      bool stopped = false;
      if (fp.rpart_prev != nullptr) {
        // the stop rule for iteration t - 1, whose residual partials the previous
        // launch wrote: every block sums them in the same order and takes the same
        // tolerance decision; block 0 advances the state (the stall rule, which
        // depends on earlier iterations, is decided there alone: a block that
        // carries on only forms w_t, which the result w_{t-1} does not share a
        // buffer with, and the next launch sees the solve done)
        if (lead) stopped = state_advance_from(st, snap, rprev);
        if (rprev < tol) return;
      }
      const double nu = (norm == NORM_L2) ? sqrt(tot) : tot;
      // block 0's thread 0 records nu_t unless it has just stopped the solve (stall rule)
      const bool owner = lead && !stopped;
      if (owner) st->nu = nu;
      if (!(nu > 0.0) || !(nu < INFINITY)) {
        if (owner) {
          st->status = MAPI_ERR_DEGENERATE;
          st->iter = fp.iter - 1;
          st->done = 1;
        }
        return;
      }
      inv = 1.0 / nu;
      if (e0 + threadIdx.x < e1) {
        const float wn = (float)((double)ys * inv);
        fp.w_new[e0 + threadIdx.x] = wn;
        racc = fabs((double)wn - (double)wo);
      }
      for (int64_t i = e0 + threadIdx.x + blockDim.x; i < e1; i += blockDim.x) {
        const float wn = (float)((double)fp.y_prev[i] * inv);
        fp.w_new[i] = wn;
        racc += fabs((double)wn - (double)fp.w_old[i]);
      }
    }
    const int64_t wfl = dense_lds_w_floats(DT, n_cols);
    // whole vectors' w in chunk-interleaved order (|w| with PF, plus one sign word
    // per 4 columns in natural order after the staged region and the tail)
    auto stage = [&](int k, float4 t) {
      if (fused)
        t = make_float4((float)((double)t.x * inv), (float)((double)t.y * inv), (float)((double)t.z * inv),
                        (float)((double)t.w * inv));
      if constexpr (PF) {
        uint32_t* sm = reinterpret_cast<uint32_t*>(w_lds + wfl + kDenseTailFloats);
        sm[k] = (sign_bit(t.x) >> 24) | (sign_bit(t.y) >> 16) | (sign_bit(t.z) >> 8) | sign_bit(t.w);
        t = make_float4(fabsf(t.x), fabsf(t.y), fabsf(t.z), fabsf(t.w));
      }
      reinterpret_cast<float4*>(w_lds)[perm_base<DT>(k / (VE / 4)) + (k % (VE / 4)) * 64] = t;
    };
    int k0 = threadIdx.x;
    if (!fused) issue_first();
    if (fused) {
#pragma unroll
      for (int q = 0; q < PQ; ++q) {
        const int k = threadIdx.x + q * blockDim.x;
        if (k < np4) stage(k, pre[q]);
      }
      k0 = threadIdx.x + PQ * blockDim.x;
    }
    // the rest in batches of PQ float4s per thread, every load of a batch issued before
    // its first store (a block of 256 threads stages half of a 16384-float w here)
    for (int kb = k0; kb < np4; kb += PQ * blockDim.x) {
      float4 t[PQ];
#pragma unroll
      for (int q = 0; q < PQ; ++q) {
        const int k = kb + q * blockDim.x;
        t[q] = k < np4 ? src[k] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int q = 0; q < PQ; ++q) {
        const int k = kb + q * blockDim.x;
        if (k < np4) stage(k, t[q]);
      }
    }
    if (fused) {   // the tail cannot be read from w: it is formed here, after the staged vectors
      float* tl = w_lds + wfl;
      for (int j = nvec * VE + threadIdx.x; j < n_cols; j += blockDim.x)
        tl[j - nvec * VE] = (float)((double)fp.y_prev[j] * inv);
      wtail = tl - nvec * VE;
    }
    __syncthreads();
    wv = w_lds;
    if constexpr (PF) smask = reinterpret_cast<const uint32_t*>(w_lds + wfl + kDenseTailFloats);
  }

  double nrm = 0.0;

  // rev: the row groups in mirrored order, so that a sweep starts where the one before
  // it (in forward order) ended; the rows each block owns change, the row sums do not
  for (int g0 = blockIdx.x * nw + wave; g0 < ngroups; g0 += gridDim.x * nw) {
    const int g = rev ? ngroups - 1 - g0 : g0;
    if (!MAPI_DCHECK(st, g >= 0 && (int64_t)g * RW < n_rows, 1)) continue;
    const bool fst = kAhead && have_first;   // the first group only
    have_first = false;
    const unsigned char* rp[RW];
    float sc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int row = min(g * RW + r, n_rows - 1);     // padded rows re-read the last row
      rp[r] = A + (int64_t)row * ld_bytes;
      sc[r] = (DT == MAPI_FP8_E4M3) ? rscale[row] : 1.0f;
    }
    float sums[RW];
    if constexpr (DT == MAPI_FP8_E4M3) {
      bool p2 = true;
#pragma unroll
      for (int r = 0; r < RW; ++r) p2 = p2 && pow2_scale(sc[r]);
      if (p2) rows_product<DT, OP, RW, U, NT, PF, true, WLDS, 1>(rp, sc, wv, n_cols, lane, sums, smask, wtail, first, fst, rot_step(g * RW, S));
      else rows_product<DT, OP, RW, U, NT, PF, false, WLDS, 1>(rp, sc, wv, n_cols, lane, sums, smask, wtail, first, fst, rot_step(g * RW, S));
    } else {
      rows_product<DT, OP, RW, U, NT, PF, false, WLDS, 1>(rp, sc, wv, n_cols, lane, sums, smask, wtail, first, fst, rot_step(g * RW, S));
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const float s = sums[r];
      const int row = g * RW + r;
      if (lane == 0 && row < n_rows) {
        y[row] = s;
        nrm += (norm == NORM_L2) ? (double)s * (double)s : fabs((double)s);
      }
    }
  }

  // One partial of the normaliser per block; the normalisation kernel that
  // follows sums them in block order (no grid-wide atomics here).
  if (part == nullptr || norm == NORM_NONE) return;
  const double bsum = block_sum_f64(nrm, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = bsum;
  if (WLDS && fp.rpart_out != nullptr) {
    const double rsum = block_sum_f64(racc, sh);
    if (threadIdx.x == 0) fp.rpart_out[blockIdx.x] = rsum;
  }
}

template <int DT, int OP, int RW, int U, int WL, bool NT>
static hipError_t launch_k(const DenseArgs& a, const float* w, float* y, double* part, SolveState* st, int norm,
                           int blocks, int waves, hipStream_t s, const FusedPrev* fp) {
  const FusedPrev f = fp ? *fp : FusedPrev{nullptr, nullptr, 0, nullptr, 0, nullptr, nullptr, nullptr};
  const unsigned char* A = static_cast<const unsigned char*>(a.A);
  const int64_t ldb = a.ld * Traits<DT>::ESZ;
  const size_t lds = dense_lds_bytes(DT, a.n_cols, WL);
  if (a.ev_start) {
    hipExtLaunchKernelGGL((k_mavp_dense<DT, OP, RW, U, WL, NT>), dim3(blocks), dim3(waves * kWave), (uint32_t)lds, s,
                          a.ev_start, a.ev_stop, 0u, A, ldb, (int)a.n_rows, (int)a.n_cols, a.row_scale, w, y, part,
                          st, norm, f, a.reverse);
  } else {
    hipLaunchKernelGGL((k_mavp_dense<DT, OP, RW, U, WL, NT>), dim3(blocks), dim3(waves * kWave), lds, s, A, ldb,
                       (int)a.n_rows, (int)a.n_cols, a.row_scale, w, y, part, st, norm, f, a.reverse);
  }
  return hipGetLastError();
}

template <int DT, int OP, int RW, int U, int WL>
static hipError_t launch_nt(const DenseArgs& a, const float* w, float* y, double* part, SolveState* st, int norm,
                            const DenseTuning& t, int blocks, hipStream_t s, const FusedPrev* fp) {
  return t.nontemporal ? launch_k<DT, OP, RW, U, WL, true>(a, w, y, part, st, norm, blocks, t.waves, s, fp)
                       : launch_k<DT, OP, RW, U, WL, false>(a, w, y, part, st, norm, blocks, t.waves, s, fp);
}

template <int DT, int OP, int RW, int U>
static hipError_t launch_wl(const DenseArgs& a, const float* w, float* y, double* part, SolveState* st, int norm,
                            const DenseTuning& t, int blocks, hipStream_t s, const FusedPrev* fp) {
  switch (t.w_in_lds) {
    case 0:
      if (fp) return hipErrorInvalidValue;   // forming w needs it staged in LDS
      return launch_nt<DT, OP, RW, U, 0>(a, w, y, part, st, norm, t, blocks, s, fp);
    case 1: return launch_nt<DT, OP, RW, U, 1>(a, w, y, part, st, norm, t, blocks, s, fp);
    case 2:
      if constexpr (DT == MAPI_FP8_E4M3) return launch_nt<DT, OP, RW, U, 2>(a, w, y, part, st, norm, t, blocks, s, fp);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <int DT, int OP, int RW>
static hipError_t launch_rw(const DenseArgs& a, const float* w, float* y, double* part, SolveState* st, int norm,
                            const DenseTuning& t, int blocks, hipStream_t s, const FusedPrev* fp) {
  return t.unroll == 4 ? launch_wl<DT, OP, RW, 4>(a, w, y, part, st, norm, t, blocks, s, fp)
                       : launch_wl<DT, OP, RW, 2>(a, w, y, part, st, norm, t, blocks, s, fp);
}

template <int DT, int OP>
static hipError_t launch_op(const DenseArgs& a, const float* w, float* y, double* part, SolveState* st, int norm,
                            const DenseTuning& t, int blocks, hipStream_t s, const FusedPrev* fp) {
  switch (t.rows_per_wave) {
    case 1: return launch_rw<DT, OP, 1>(a, w, y, part, st, norm, t, blocks, s, fp);
    case 2: return launch_rw<DT, OP, 2>(a, w, y, part, st, norm, t, blocks, s, fp);
    case 4: return launch_rw<DT, OP, 4>(a, w, y, part, st, norm, t, blocks, s, fp);
    case 8: return launch_rw<DT, OP, 8>(a, w, y, part, st, norm, t, blocks, s, fp);
    default: return hipErrorInvalidValue;
  }
}

template <int DT>
static hipError_t launch_dt(const DenseArgs& a, int op, const float* w, float* y, double* part, SolveState* st,
                            int norm, const DenseTuning& t, int blocks, hipStream_t s, const FusedPrev* fp) {
  switch (op) {
    case MAPI_OP_MIN1: return launch_op<DT, MAPI_OP_MIN1>(a, w, y, part, st, norm, t, blocks, s, fp);
    case MAPI_OP_MIN2: return launch_op<DT, MAPI_OP_MIN2>(a, w, y, part, st, norm, t, blocks, s, fp);
    case MAPI_OP_DIAMOND: return launch_op<DT, MAPI_OP_DIAMOND>(a, w, y, part, st, norm, t, blocks, s, fp);
    case MAPI_OP_DOT: return launch_op<DT, MAPI_OP_DOT>(a, w, y, part, st, norm, t, blocks, s, fp);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mapi
