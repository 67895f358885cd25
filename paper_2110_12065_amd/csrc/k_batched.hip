// Persistent batched kernel: ragged MAPI / RPI instances (dense float32, bf16 or
// fp8 storage, device-generated dense matrices, CSR PageRank) iterated to
// convergence by one long-lived grid that pops (instance, phase, tile) items
// from a device work queue.
//
// Per instance the phases are: GEN (generated matrices only) -> INIT (start
// vector, PageRank scalars) -> { PROD (product rows and the normaliser's
// partial) -> FIN (normalise, residual, stop rule) } * -> OUT (copy the result).
// The block that completes the last tile of a phase reduces the partials in
// tile order and pushes the next phase, so an instance's arithmetic does not
// depend on which block ran which tile or on what else is in the batch.
// Instances whose product is one tile run whole iterations inside one block,
// and the block that completes a phase of a one-tile vector runs the next step
// itself instead of queueing it.
#include <hip/hip_runtime.h>

#include "batched.h"
#include "dense_kernel.h"

namespace mapi {

constexpr int kBT = 256;   // threads per block

__device__ __forceinline__ int64_t now_ticks() { return (int64_t)__builtin_amdgcn_s_memrealtime(); }

// ---------------------------------------------------------------- queue
// A consumer claims a position with one fetch-add of `head` (no retry loop, so
// claims do not serialise under contention) and polls that position's slot with
// relaxed loads: on gfx950 an agent-scope acquire invalidates the XCD's L2, so
// only a block that has its item acquires, once.  A block that publishes
// results releases once (one fence by one thread after the block barrier).

__device__ __forceinline__ unsigned long long* q_slot(BQueue* q, unsigned long long p) {
  return &q->item[p & q->mask];
}
__device__ __forceinline__ bool slot_is(unsigned long long v, unsigned long long p) {
  return (v >> kTagShift) == ((p + 1) & 0x1FFFFFFull);
}
__device__ __forceinline__ unsigned long long slot_load(const unsigned long long* s) {
  return __hip_atomic_load(const_cast<unsigned long long*>(s), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Write `item` at position p; if p's consumer has already given p up, write it at
// a newly reserved position instead.  Terminates: each skipped position belongs
// to a block that has left.
__device__ void q_put(BQueue* q, unsigned long long p, unsigned long long item) {
  for (;;) {
    unsigned long long* s = q_slot(q, p);
    unsigned long long old = slot_load(s);
    while (!slot_is(old, p))
      if (__hip_atomic_compare_exchange_strong(s, &old, bslot(p, item), __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT))
        return;
    p = atomicAdd(&q->tail, 1ull);
  }
}

// Push `count` tiles of one phase; called by every thread of the block after
// the block's results are written.
__device__ void q_push(BQueue* q, uint32_t inst, int phase, uint32_t count, unsigned long long* sh_base) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();   // release this block's results
    *sh_base = atomicAdd(&q->tail, (unsigned long long)count);
  }
  __syncthreads();
  const unsigned long long base = *sh_base;
  for (uint32_t t = threadIdx.x; t < count; t += blockDim.x) q_put(q, base + t, bitem(inst, phase, t));
  __syncthreads();
}

// Serving: move newly submitted items from the host inbox into the queue (block 0, thread 0).
__device__ void drain_inbox(BQueue* q, BCtl* ctl) {
  const unsigned long long tail = *ctl->inbox_tail;
  unsigned long long h = ctl->inbox_head;
  if (h == tail) return;
  __threadfence_system();
  const unsigned long long base = atomicAdd(&q->tail, tail - h);
  for (unsigned long long k = 0; h < tail; ++h, ++k) {
    const unsigned long long v = ctl->inbox[h & ctl->inbox_mask];
    if (item_phase(v) == PH_ADMIT) {
      atomicAdd(&q->live, 1u);   // a newly admitted instance: counted before its item is visible
      __threadfence();
    }
    q_put(q, base + k, v);
  }
  ctl->inbox_head = h;
  *ctl->inbox_head_host = h;
  __threadfence_system();
}

// Wait for the item of position p (thread 0).  Returns false when the block
// should leave; p is then marked skipped, unless its item arrived first.
__device__ bool q_take(BQueue* q, const BInst* insts, BCtl* ctl, unsigned long long p, int64_t deadline,
                       unsigned long long* out) {
  unsigned long long* s = q_slot(q, p);
  const int64_t t0 = now_ticks();
  for (int polls = 0;; ++polls) {
    if (ctl->mode == 1 && blockIdx.x == 0) drain_inbox(q, ctl);
    unsigned long long v = slot_load(s);
    if (!slot_is(v, p)) {
      const int64_t now = now_ticks();
      const uint32_t live = __hip_atomic_load(&q->live, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      bool leave = false;
      if (now > deadline) {
        if (live) atomicOr(&q->error, 1u);
        leave = true;
      } else if (live == 0 && (ctl->mode == 0 || *ctl->quit)) {
        leave = true;
      } else if (now - t0 > ctl->idle_limit && !(ctl->mode == 1 && blockIdx.x == 0 && live)) {
        leave = true;   // block 0 drains the serving inbox: it stays while admitted work is live
      }
      if (!leave) {
        if (polls < 16) __builtin_amdgcn_s_sleep(2);
        else __builtin_amdgcn_s_sleep(32);
        continue;
      }
      if (__hip_atomic_compare_exchange_strong(s, &v, bslot(p, bitem(0, PH_SKIP, 0)), __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        return false;
      // the item arrived meanwhile: v holds it
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // see the producer's results
    *out = v & kItemMask;
    return true;
  }
}

// Count a finished tile of the current phase; true in every thread of the block
// that finished the last one.  That block then sees every other tile's results.
__device__ bool tile_arrive(BInst* I, uint32_t tiles, int* sh_flag) {
  if (tiles == 1) {
    __syncthreads();
    return true;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();   // release this tile's results
    const uint32_t prev = atomicAdd(&I->arrive, 1u);
    const bool last = prev == tiles - 1;
    if (last) {
      __hip_atomic_store(&I->arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();   // acquire the other tiles' results
    }
    *sh_flag = last ? 1 : 0;
  }
  __syncthreads();
  return *sh_flag != 0;
}

// ---------------------------------------------------------------- row products
// Rows [r0, r1) of one tile: each wave takes RW rows at a time (4 for float32 and
// bf16 storage, 2 for FP8, whose decoded vectors need more registers) with two
// 16-byte loads per row and lane in flight.
// WSP: 3 when w was staged in LDS, 1 when it is read from device memory.
template <int DT, int OP, int WSP>
__device__ double dense_rows_t(const BInst* I, const float* wv, int r0, int r1, float* y, bool l2) {
  constexpr int RW = (DT == MAPI_FP8_E4M3) ? 2 : 4;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
  const unsigned char* A = static_cast<const unsigned char*>(I->A);
  const int64_t ldb = I->ld * Traits<DT>::ESZ;
  const int S = I->n / Traits<DT>::VE / kWave;   // whole wave-steps of a row
  double nrm = 0.0;
  if (!MAPI_DCHECK(&I->st, r0 >= 0 && r1 <= I->n, 4)) return 0.0;   // a row tile outside the matrix
  for (int g = r0 + RW * wave; g < r1; g += RW * nw) {
    const unsigned char* rp[RW];
    float sc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int row = min(g + r, r1 - 1);   // padded rows re-read the tile's last row
      rp[r] = A + (int64_t)row * ldb;
      sc[r] = (DT == MAPI_FP8_E4M3) ? I->row_scale[row] : 1.0f;
    }
    float s[RW];
    const uint4 none[2][RW] = {};   // no step loaded ahead here
    if constexpr (DT == MAPI_FP8_E4M3) {
      bool p2 = true;
#pragma unroll
      for (int r = 0; r < RW; ++r) p2 = p2 && pow2_scale(sc[r]);
      if (p2) rows_product<DT, OP, RW, 2, false, false, true, false, WSP>(rp, sc, wv, I->n, lane, s, nullptr, nullptr, none, false, rot_step(g, S));
      else rows_product<DT, OP, RW, 2, false, false, false, false, WSP>(rp, sc, wv, I->n, lane, s, nullptr, nullptr, none, false, rot_step(g, S));
    } else {
      rows_product<DT, OP, RW, 2, false, false, false, false, WSP>(rp, sc, wv, I->n, lane, s, nullptr, nullptr, none, false, rot_step(g, S));
    }
#pragma unroll
    for (int r = 0; r < RW; ++r)
      if (lane == 0 && g + r < r1) {
        y[g + r] = s[r];
        nrm += l2 ? (double)s[r] * (double)s[r] : fabs((double)s[r]);
      }
  }
  return nrm;
}

template <int DT, int WSP>
__device__ double dense_rows_op(const BInst* I, int op, const float* wv, int r0, int r1, float* y, bool l2) {
  switch (op) {
    case MAPI_OP_MIN2: return dense_rows_t<DT, MAPI_OP_MIN2, WSP>(I, wv, r0, r1, y, l2);
    case MAPI_OP_DOT: return dense_rows_t<DT, MAPI_OP_DOT, WSP>(I, wv, r0, r1, y, l2);
    default: return dense_rows_t<DT, MAPI_OP_MIN1, WSP>(I, wv, r0, r1, y, l2);
  }
}

// w in LDS (stage_w staged it: n fits) or in device memory, each read in its own
// address space
template <int DT>
__device__ double dense_rows_w(const BInst* I, int op, const float* wv, int r0, int r1, float* y, bool l2) {
  if (I->n <= kBatchLdsFloats) return dense_rows_op<DT, 3>(I, op, wv, r0, r1, y, l2);
  return dense_rows_op<DT, 1>(I, op, wv, r0, r1, y, l2);
}

__device__ double dense_rows(const BInst* I, const float* wv, int r0, int r1, float* y) {
  const bool rpi = I->method == MAPI_METHOD_RPI;
  const int op = rpi ? MAPI_OP_DOT : I->op;
  switch (I->dtype) {
    case MAPI_BF16: return dense_rows_w<MAPI_BF16>(I, op, wv, r0, r1, y, rpi);
    case MAPI_FP8_E4M3: return dense_rows_w<MAPI_FP8_E4M3>(I, op, wv, r0, r1, y, rpi);
    default: return dense_rows_w<MAPI_F32>(I, op, wv, r0, r1, y, rpi);
  }
}

// PageRank rows (eq. 11 split sums, as in the single-solve kernel): G lanes per
// row, each lane summing the row's in-links k = sub, sub + G, ... in order, then a
// fixed butterfly.  Each lane group carries R rows at once, so a lane has R
// independent index, value and gather loads in flight per step: the persistent
// kernel runs few waves per SIMD and must hide the gathers' latency itself.
__device__ double csr_rows(const BInst* I, const float* w, int r0, int r1, float* y) {
  constexpr int G = 8, R = 4;
  const bool mapi = I->method == MAPI_METHOD_MAPI;
  const double base = mapi ? I->st.ex[0] + I->st.ex[1]
                           : ((double)I->alpha * I->inv_n) * I->st.ex[1] + (double)I->c * I->st.ex[0];
  const float alpha = I->alpha, c = I->c;
  const int32_t* __restrict__ row_ptr = I->row_ptr;
  const int32_t* __restrict__ col = I->col;
  const float* __restrict__ val = I->val;
  const int sub = threadIdx.x % G, grp = threadIdx.x / G, ngrp = blockDim.x / G;
  double nrm = 0.0;
  for (int i0 = r0 + grp * R; i0 < r1; i0 += ngrp * R) {
    int32_t p0[R], len[R];
    int32_t maxlen = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool ok = i0 + r < r1;
      p0[r] = ok ? row_ptr[i0 + r] : 0;
      len[r] = ok ? row_ptr[i0 + r + 1] - p0[r] : 0;
      maxlen = max(maxlen, len[r]);
    }
    float acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0f;
    for (int32_t k = sub; k < maxlen; k += G) {
      int32_t cj[R];
      float h[R], wj[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool ok = k < len[r];
        cj[r] = ok ? col[p0[r] + k] : 0;
        h[r] = ok ? val[p0[r] + k] : 0.0f;
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (!MAPI_DCHECK(&I->st, (uint32_t)cj[r] < (uint32_t)I->n, 4)) cj[r] = 0;   // a source outside 0..n-1
        wj[r] = w[cj[r]];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (k < len[r]) {
          if (mapi) {
            const float g = fmaf(alpha, h[r], c);
            acc[r] += __builtin_amdgcn_fmed3f(wj[r], -g, g) - __builtin_amdgcn_fmed3f(wj[r], -c, c);
          } else {
            acc[r] = fmaf(h[r], wj[r], acc[r]);
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      float a = acc[r];
#pragma unroll
      for (int off = G / 2; off >= 1; off >>= 1) a += __shfl_xor(a, off, G);
      if (sub == 0 && i0 + r < r1) {
        const float yi = mapi ? (float)(base + (double)a) : (float)((double)alpha * (double)a + base);
        y[i0 + r] = yi;
        nrm += fabs((double)yi);
      }
    }
  }
  return nrm;
}

// Stage w in LDS; every thread issues all its loads before its first store, so
// the staging costs one memory latency rather than one per pass.
__device__ const float* stage_w(const BInst* I, const float* w, float* lds) {
  if (I->kind == BK_CSR || I->n > kBatchLdsFloats) return w;
  constexpr int K = kBatchLdsFloats / 4 / kBT;
  const int n = I->n, nv4 = n >> 2;
  float4 t[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int v = threadIdx.x + k * kBT;
    if (v < nv4) t[k] = reinterpret_cast<const float4*>(w)[v];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int v = threadIdx.x + k * kBT;
    if (v < nv4) reinterpret_cast<float4*>(lds)[v] = t[k];
  }
  for (int j = (nv4 << 2) + threadIdx.x; j < n; j += kBT) lds[j] = w[j];
  __syncthreads();
  return lds;
}

// Normalise rows [r0, r1) of y by nu into w_new; returns the residual and PageRank
// partials.  Each thread visits i = r0 + tid, r0 + tid + kBT, ... in order, with the
// loads of four visits issued ahead of their use.
__device__ void fin_rows(const BInst* I, const float* y, const float* w_old, float* w_new, int r0, int r1, double nu,
                         double* r, double* e0, double* e1) {
  constexpr int U = 4;
  const double c = (double)I->c;
  const double inv_n = I->inv_n;
  const bool csr = I->kind == BK_CSR, mapi = I->method == MAPI_METHOD_MAPI;
  const uint8_t* dangling = I->dangling;
  for (int i0 = r0 + (int)threadIdx.x; i0 < r1; i0 += U * kBT) {
    float yv[U], wo[U];
    uint8_t dg[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * kBT;
      const bool ok = i < r1;
      yv[u] = ok ? y[i] : 0.0f;
      wo[u] = ok ? w_old[i] : 0.0f;
      dg[u] = (ok && csr) ? dangling[i] : (uint8_t)0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * kBT;
      if (i >= r1) break;
      const float wn = (float)((double)yv[u] / nu);
      w_new[i] = wn;
      const double wd = (double)wn;
      *r += fabs(wd - (double)wo[u]);
      if (csr) {
        if (mapi) {
          const double tc = fmin(fmax(wd, -c), c);
          *e0 += tc;
          if (dg[u]) *e1 += fmin(fmax(wd, -inv_n), inv_n) - tc;
        } else {
          *e0 += wd;
          if (dg[u]) *e1 += wd;
        }
      }
    }
  }
}

__device__ __forceinline__ bool bad_norm(double nu) { return !(nu > 0.0) || !(nu < INFINITY); }

// ---------------------------------------------------------------- phases
__device__ void phase_gen(BInst* I, uint32_t tile) {
  const int n = I->n;
  const int r0 = tile * kGenRows, r1 = min(n, r0 + kGenRows);
  const uint64_t base = splitmix64(I->seed), sbase = splitmix64(I->seed ^ 0x5BD1E995ull);
  void* A = const_cast<void*>(I->A);
  if (I->dtype == MAPI_BF16) gen_rows<true>(A, I->ld, n, r0, r1, base, sbase, I->gen_scale, I->gen_spike);
  else gen_rows<false>(A, I->ld, n, r0, r1, base, sbase, I->gen_scale, I->gen_spike);
}

// Start vector rows; PageRank scalars of w0 into part.
__device__ void phase_init(BInst* I, uint32_t tile, double* sh) {
  const int n = I->n;
  const int r0 = tile * kVecTile, r1 = min(n, r0 + kVecTile);
  const uint64_t vbase = splitmix64(I->seed ^ 0x1B873593ull);
  const float inv_sqrt_n = I->gen_w0;
  double e0 = 0.0, e1 = 0.0;
  const double c = (double)I->c, inv_n = I->inv_n;
  for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    float v;
    if (I->w0) v = I->w0[i];
    else if (I->kind == BK_CSR) v = (float)inv_n;
    else v = (splitmix64(vbase + (uint64_t)i) >> 63) ? -inv_sqrt_n : inv_sqrt_n;   // unit l2 norm
    I->wb0[i] = v;
    if (I->kind == BK_CSR) {
      const double wd = (double)v;
      if (I->method == MAPI_METHOD_MAPI) {
        const double tc = fmin(fmax(wd, -c), c);
        e0 += tc;
        if (I->dangling[i]) e1 += fmin(fmax(wd, -inv_n), inv_n) - tc;
      } else {
        e0 += wd;
        if (I->dangling[i]) e1 += wd;
      }
    }
  }
  e0 = block_sum_f64(e0, sh);
  e1 = block_sum_f64(e1, sh);
  if (threadIdx.x == 0) {
    store_agent(&I->part[I->ntiles + 3 * tile + 1], e0);
    store_agent(&I->part[I->ntiles + 3 * tile + 2], e1);
  }
}

// Normalise the whole iterate by nu, then residual and stop rule, by one block
// (instances whose vectors are one tile).  Returns whether the solve is done.
__device__ bool fin_whole(BInst* I, double nu, double* sh) {
  const int it = I->st.iter;
  const float* wc = (it & 1) ? I->wb1 : I->wb0;
  float* wn = (it & 1) ? I->wb0 : I->wb1;
  double r = 0.0, e0 = 0.0, e1 = 0.0;
  const bool bad = bad_norm(nu);
  if (!bad) fin_rows(I, I->y, wc, wn, 0, I->n, nu, &r, &e0, &e1);
  r = block_sum_f64(r, sh);
  e0 = block_sum_f64(e0, sh);
  e1 = block_sum_f64(e1, sh);
  if (threadIdx.x == 0) {
    I->st.nu = nu;
    if (bad) {
      I->st.status = MAPI_ERR_DEGENERATE;
      I->st.done = 1;
    } else {
      I->st.ex[0] = e0;
      I->st.ex[1] = e1;
      state_advance(&I->st, r);
    }
  }
  __threadfence_block();
  __syncthreads();
  return I->st.done != 0;
}

// One block iterates a one-tile instance: product, normaliser, normalisation,
// residual, stop rule, up to kSoloBurst times.  Returns whether it is done.
__device__ bool phase_solo(BInst* I, float* lds, double* sh) {
  const int n = I->n;
  const bool rpi = I->method == MAPI_METHOD_RPI;
  for (int k = 0; k < kSoloBurst; ++k) {
    const float* wc = (I->st.iter & 1) ? I->wb1 : I->wb0;
    double nrm;
    if (I->kind == BK_CSR) {
      nrm = csr_rows(I, wc, 0, n, I->y);
    } else {
      const float* wv = stage_w(I, wc, lds);
      nrm = dense_rows(I, wv, 0, n, I->y);
    }
    double nu = block_sum_f64(nrm, sh);
    if (rpi && I->kind != BK_CSR) nu = sqrt(nu);
    __threadfence_block();
    __syncthreads();
    if (fin_whole(I, nu, sh)) return true;
  }
  return false;
}

// Copy rows [r0, r1) of the final iterate to the caller's output.
__device__ void out_rows(const BInst* I, int r0, int r1) {
  constexpr int U = 4;
  const float* src = (I->st.iter & 1) ? I->wb1 : I->wb0;
  float* out = I->out;
  for (int i0 = r0 + (int)threadIdx.x; i0 < r1; i0 += U * kBT) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = (i0 + u * kBT < r1) ? src[i0 + u * kBT] : 0.0f;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u * kBT < r1) out[i0 + u * kBT] = v[u];
  }
  __threadfence_system();
}

// Retire a finished instance (after every output tile is written): completion
// record for the server, then one instance fewer live.
__device__ void retire(BInst* I, uint32_t ii, BQueue* q, BCtl* ctl) {
  __syncthreads();
  if (threadIdx.x == 0) {
    I->t_done = now_ticks();
    if (ctl->mode == 1) {
      const unsigned long long p = atomicAdd(&ctl->done_pos, 1ull);
      BDone* d = ctl->done + (p & ctl->done_mask);
      d->slot = (int32_t)ii;
      d->slot_gen = I->slot_gen;
      d->status = I->st.status;
      d->iters = I->st.iter;
      d->converged = I->st.converged;
      d->residual = I->st.r;
      d->norm = I->st.nu;
      d->t_admit = I->t_admit;
      d->t_start = I->t_start;
      d->t_done = I->t_done;
      __threadfence_system();
      __hip_atomic_store(&d->seq, p + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __threadfence();
    atomicSub(&q->live, 1u);
  }
  __syncthreads();
}

struct Shared {
  double sh[16];
  unsigned long long base;
  int flag;
};

// Continue an instance whose state this block has just brought up to date: a
// one-tile instance runs its next burst here; a finished one writes its output
// (here when it is one tile, else as queued tiles); otherwise its next product
// phase is queued.
__device__ void advance(BQueue* q, BInst* I, uint32_t ii, BCtl* ctl, float* lds, Shared* S) {
  if (!I->st.done && I->solo && !phase_solo(I, lds, S->sh)) {
    q_push(q, ii, PH_PROD, 1u, &S->base);
    return;
  }
  if (I->st.done) {
    if (I->vtiles == 1) {
      out_rows(I, 0, I->n);
      retire(I, ii, q, ctl);
    } else {
      q_push(q, ii, PH_OUT, I->vtiles, &S->base);
    }
    return;
  }
  q_push(q, ii, PH_PROD, (uint32_t)I->ntiles, &S->base);
}

// Start-vector tile; the block that completes the last one starts the iterations.
__device__ void run_init(BQueue* q, BInst* I, uint32_t ii, uint32_t tile, BCtl* ctl, float* lds, Shared* S) {
  phase_init(I, tile, S->sh);
  if (!tile_arrive(I, I->vtiles, &S->flag)) return;
  const double E0 = block_sum_parts(I->part + I->ntiles, I->vtiles, 3, 1, S->sh);
  const double E1 = block_sum_parts(I->part + I->ntiles, I->vtiles, 3, 2, S->sh);
  if (threadIdx.x == 0) {
    I->st.ex[0] = E0;
    I->st.ex[1] = E1;
    if (I->max_iters <= 0) I->st.done = 1;
  }
  __threadfence_block();
  __syncthreads();
  advance(q, I, ii, ctl, lds, S);
}

// ---------------------------------------------------------------- admission (serving)
// A served request reaches the device as one ADMIT item: its descriptor is read
// from pinned host memory, and a PageRank request's CSR arrays are read from the
// caller's pinned host memory by the PREP phases, so admission needs no copy
// command or kernel beside the persistent kernel.

// End an instance without solving it (invalid input found on the device).
__device__ void reject(BInst* I, uint32_t ii, BQueue* q, BCtl* ctl, int status) {
  if (threadIdx.x == 0) {
    I->st.status = status;
    I->st.done = 1;
  }
  retire(I, ii, q, ctl);
}

// First phase of an admitted instance: CSR checks, generation, or the start vector.
__device__ void start_instance(BQueue* q, BInst* I, uint32_t ii, BCtl* ctl, float* lds, Shared* S);

__device__ void phase_admit(BQueue* q, BInst* insts, uint32_t ii, BCtl* ctl, float* lds, Shared* S) {
  BInst* I = insts + ii;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(ctl->inst_stage + ii);
  uint32_t* dst = reinterpret_cast<uint32_t*>(I);
  for (int k = threadIdx.x; k < (int)(sizeof(BInst) / 4); k += kBT) dst[k] = src[k];
  __threadfence_block();
  __syncthreads();
  start_instance(q, I, ii, ctl, lds, S);
}

__device__ void start_instance(BQueue* q, BInst* I, uint32_t ii, BCtl* ctl, float* lds, Shared* S) {
  if (threadIdx.x == 0) I->t_start = now_ticks();
  if (I->kind == BK_CSR && I->src_row_ptr) q_push(q, ii, PH_PREPA, (uint32_t)I->vtiles, &S->base);
  else if (I->kind == BK_GEN) q_push(q, ii, PH_GEN, (uint32_t)I->gtiles, &S->base);
  else q_push(q, ii, PH_INIT, (uint32_t)I->vtiles, &S->base);
}

// Rows [r0, r1) of a served CSR request: copy row_ptr (and its last entry), check it,
// mark every node dangling (PREPB clears the ones that are sources).
__device__ void phase_prepa(BInst* I, uint32_t tile) {
  const int n = I->n;
  const int r0 = tile * kVecTile, r1 = min(n, r0 + kVecTile);
  const int32_t* src = I->src_row_ptr;
  int32_t* rp = const_cast<int32_t*>(I->row_ptr);
  uint8_t* dg = const_cast<uint8_t*>(I->dangling);
  uint32_t err = 0;
  for (int i = r0 + threadIdx.x; i < r1; i += kBT) {
    const int32_t a = src[i], b = src[i + 1];
    rp[i] = a;
    dg[i] = 1;
    if (a > b) err |= 2u;
    if (i == 0 && a != 0) err |= 1u;
    if (i == n - 1) {
      rp[n] = b;
      if ((int64_t)b != I->nnz) err |= 1u;
    }
  }
  if (err) atomicOr(&I->prep_err, err);
}

// Links [p0, p1): copy col and val, check the column range, clear the dangling
// flag of every source (the same byte may be cleared by several threads).
__device__ void phase_prepb(BInst* I, uint32_t tile) {
  const int64_t p0 = (int64_t)tile * kEdgeTile, p1 = min(I->nnz, p0 + kEdgeTile);
  const int n = I->n;
  int32_t* col = const_cast<int32_t*>(I->col);
  float* val = const_cast<float*>(I->val);
  uint8_t* dg = const_cast<uint8_t*>(I->dangling);
  uint32_t err = 0;
  constexpr int U = 4;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += U * kBT) {
    int32_t j[U];
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = p + u * kBT;
      j[u] = e < p1 ? I->src_col[e] : 0;
      v[u] = e < p1 ? I->src_val[e] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = p + u * kBT;
      if (e >= p1) break;
      col[e] = j[u];
      val[e] = v[u];
      if (j[u] < 0 || j[u] >= n) err |= 4u;
      else dg[j[u]] = 0;
    }
  }
  if (err) atomicOr(&I->prep_err, err);
}

__device__ __forceinline__ uint32_t prep_error(BInst* I) {
  return __hip_atomic_load(&I->prep_err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Two blocks (8 waves) per compute unit, at most 256 VGPRs: the kernel holds every
// phase's code, and at 128 VGPRs (four blocks) it spilled to scratch; without the
// spills and with half the blocks claiming items, the generated mixes ran 6-12 % faster.
#ifndef MAPI_PERSIST_MIN_BLOCKS
#define MAPI_PERSIST_MIN_BLOCKS 2
#endif
__global__ void __launch_bounds__(kBT, MAPI_PERSIST_MIN_BLOCKS) k_persistent(BQueue* q, BInst* insts, BCtl* ctl) {
  __shared__ float4 lds4[kBatchLdsFloats / 4];
  __shared__ Shared S;
  __shared__ unsigned long long sh_item;
  __shared__ int sh_ok;
  float* lds = reinterpret_cast<float*>(lds4);
  double* sh = S.sh;
  const int64_t deadline = now_ticks() + ctl->run_limit;

  for (;;) {
    if (threadIdx.x == 0) {
      unsigned long long v = 0;
      bool ok = false;
      if (now_ticks() <= deadline) ok = q_take(q, insts, ctl, atomicAdd(&q->head, 1ull), deadline, &v);
      sh_ok = ok ? 1 : 0;
      sh_item = v;
    }
    __syncthreads();
    if (!sh_ok) return;
    const unsigned long long item = sh_item;
    const uint32_t ii = item_inst(item);
    const int ph = item_phase(item);
    const uint32_t tile = item_tile(item);
    BInst* I = insts + ii;
    const int n = I->n;

    if (ph == PH_GEN) {
      if (threadIdx.x == 0 && tile == 0 && ctl->mode == 0) I->t_start = now_ticks();
      phase_gen(I, tile);
      if (tile_arrive(I, I->gtiles, &S.flag)) {
        if (I->vtiles == 1) run_init(q, I, ii, 0, ctl, lds, &S);
        else q_push(q, ii, PH_INIT, I->vtiles, &S.base);
      }
    } else if (ph == PH_INIT) {
      if (threadIdx.x == 0 && tile == 0 && I->kind != BK_GEN && ctl->mode == 0) I->t_start = now_ticks();
      run_init(q, I, ii, tile, ctl, lds, &S);
    } else if (ph == PH_PROD) {
      if (I->solo) {
        advance(q, I, ii, ctl, lds, &S);
      } else {
        const float* wc = (I->st.iter & 1) ? I->wb1 : I->wb0;
        const int r0 = tile * I->rows_per_tile, r1 = min(n, r0 + I->rows_per_tile);
        double nrm;
        if (I->kind == BK_CSR) {
          nrm = csr_rows(I, wc, r0, r1, I->y);
        } else {
          const float* wv = stage_w(I, wc, lds);
          nrm = dense_rows(I, wv, r0, r1, I->y);
        }
        nrm = block_sum_f64(nrm, sh);
        if (threadIdx.x == 0) store_agent(&I->part[tile], nrm);
        if (tile_arrive(I, I->ntiles, &S.flag)) {
          double nu = block_sum_parts(I->part, I->ntiles, 1, 0, sh);
          if (I->method == MAPI_METHOD_RPI && I->kind != BK_CSR) nu = sqrt(nu);
          if (I->vtiles == 1) {
            fin_whole(I, nu, sh);
            advance(q, I, ii, ctl, lds, &S);
          } else {
            if (threadIdx.x == 0) I->st.nu = nu;
            q_push(q, ii, PH_FIN, I->vtiles, &S.base);
          }
        }
      }
    } else if (ph == PH_FIN) {
      const int it = I->st.iter;
      const float* wc = (it & 1) ? I->wb1 : I->wb0;
      float* wn = (it & 1) ? I->wb0 : I->wb1;
      const double nu = I->st.nu;
      double r = 0.0, e0 = 0.0, e1 = 0.0;
      if (!bad_norm(nu)) fin_rows(I, I->y, wc, wn, tile * kVecTile, min(n, (int)(tile + 1) * kVecTile), nu, &r, &e0, &e1);
      r = block_sum_f64(r, sh);
      e0 = block_sum_f64(e0, sh);
      e1 = block_sum_f64(e1, sh);
      if (threadIdx.x == 0) {
        store_agent(&I->part[I->ntiles + 3 * tile + 0], r);
        store_agent(&I->part[I->ntiles + 3 * tile + 1], e0);
        store_agent(&I->part[I->ntiles + 3 * tile + 2], e1);
      }
      if (tile_arrive(I, I->vtiles, &S.flag)) {
        const double R = block_sum_parts(I->part + I->ntiles, I->vtiles, 3, 0, sh);
        const double E0 = block_sum_parts(I->part + I->ntiles, I->vtiles, 3, 1, sh);
        const double E1 = block_sum_parts(I->part + I->ntiles, I->vtiles, 3, 2, sh);
        if (threadIdx.x == 0) {
          if (bad_norm(nu)) {
            I->st.status = MAPI_ERR_DEGENERATE;
            I->st.done = 1;
          } else {
            I->st.ex[0] = E0;
            I->st.ex[1] = E1;
            state_advance(&I->st, R);
          }
        }
        __threadfence_block();
        __syncthreads();
        advance(q, I, ii, ctl, lds, &S);
      }
    } else if (ph == PH_OUT) {
      out_rows(I, tile * kVecTile, min(n, (int)(tile + 1) * kVecTile));
      if (tile_arrive(I, I->vtiles, &S.flag)) retire(I, ii, q, ctl);
    } else if (ph == PH_ADMIT) {
      phase_admit(q, insts, ii, ctl, lds, &S);
    } else if (ph == PH_PREPA) {
      phase_prepa(I, tile);
      if (tile_arrive(I, I->vtiles, &S.flag)) {
        if (prep_error(I)) reject(I, ii, q, ctl, MAPI_ERR_ARG);
        else if (I->nnz > 0) q_push(q, ii, PH_PREPB, (uint32_t)I->etiles, &S.base);
        else if (I->vtiles == 1) run_init(q, I, ii, 0, ctl, lds, &S);
        else q_push(q, ii, PH_INIT, (uint32_t)I->vtiles, &S.base);
      }
    } else if (ph == PH_PREPB) {
      phase_prepb(I, tile);
      if (tile_arrive(I, I->etiles, &S.flag)) {
        if (prep_error(I)) reject(I, ii, q, ctl, MAPI_ERR_ARG);
        else if (I->vtiles == 1) run_init(q, I, ii, 0, ctl, lds, &S);
        else q_push(q, ii, PH_INIT, (uint32_t)I->vtiles, &S.base);
      }
    }
    __syncthreads();
  }
}

// Generated problem written out: A (float32, row pitch ld) and its start vector.
// Each block takes `rows` consecutive rows at a time.
__global__ void __launch_bounds__(256) k_gen_dense(int n, int rows, uint64_t seed, float* A, int64_t ld, float* w0,
                                                 float s_n, float spike, float inv_sqrt_n) {
  const uint64_t base = splitmix64(seed), sbase = splitmix64(seed ^ 0x5BD1E995ull);
  const uint64_t vbase = splitmix64(seed ^ 0x1B873593ull);
  for (int r0 = blockIdx.x * rows; r0 < n; r0 += gridDim.x * rows) {
    const int r1 = min(n, r0 + rows);
    gen_rows<false>(A, ld, n, r0, r1, base, sbase, s_n, spike);
    if (w0 && threadIdx.x < r1 - r0) {
      const int i = r0 + threadIdx.x;
      w0[i] = (splitmix64(vbase + (uint64_t)i) >> 63) ? -inv_sqrt_n : inv_sqrt_n;
    }
  }
}

hipError_t launch_gen_dense(int n, uint64_t seed, float* A, int64_t ld, float* w0, hipStream_t s) {
  const GenConsts g = gen_consts(n);
  // At least ~2048 blocks where n allows, up to 32 rows each (a column sign is
  // hashed once per block-row group).
  const int rows = n / 2048 < 1 ? 1 : (n / 2048 > 32 ? 32 : n / 2048);
  const int64_t groups = ((int64_t)n + rows - 1) / rows;
  const int grid = (int)(groups < 16384 ? (groups > 0 ? groups : 1) : 16384);
  hipLaunchKernelGGL(k_gen_dense, dim3(grid), dim3(256), 0, s, n, rows, seed, A, ld, w0, g.scale, g.spike, g.w0);
  return hipGetLastError();
}

// The generated problem's start vector alone: w_i = -+fl32(1 / sqrt(n)) by the top bit
// of splitmix64(splitmix64(seed ^ 0x1B873593) + i), as k_gen_dense writes it.
__global__ void __launch_bounds__(256) k_gen_start(int n, uint64_t seed, float* w, float inv_sqrt_n) {
  const uint64_t vbase = splitmix64(seed ^ 0x1B873593ull);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    w[i] = (splitmix64(vbase + (uint64_t)i) >> 63) ? -inv_sqrt_n : inv_sqrt_n;
}

hipError_t launch_gen_start(int n, uint64_t seed, float* w, hipStream_t s) {
  const int grid = (n + 255) / 256 < 1024 ? ((n + 255) / 256 > 0 ? (n + 255) / 256 : 1) : 1024;
  hipLaunchKernelGGL(k_gen_start, dim3(grid), dim3(256), 0, s, n, seed, w, gen_consts(n).w0);
  return hipGetLastError();
}

int persistent_threads() { return kBT; }

hipError_t launch_persistent(BQueue* q, BInst* inst, BCtl* ctl, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_persistent, dim3(blocks), dim3(kBT), 0, s, q, inst, ctl);
  return hipGetLastError();
}

}  // namespace mapi
