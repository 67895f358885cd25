// Mini-batch MAPI with momentum (Algorithm 3, Sec. 3.2): every run iterates, for
// t = 0 .. T-1 with the batch B_t of s sample indices,
//   A_t     = (1/s) sum_{i in B_t} x_i (+) x_i^T     (eq. 5 on the batch; float64 sums, stored float32)
//   w_{t+1} = A_t (+) w_t - beta w_{t-1}              (float32 product, w_{-1} = 0)
//   nu = ||w_{t+1}||_1 (float64);  w_t <- w_t / nu;  w_{t+1} <- w_{t+1} / nu
// and optionally divides w_T by its l2 norm.  The data matrix is N x D with the
// samples as rows (Algorithm 3's layout), so a gathered sample is one contiguous row.
//
// A_t depends on the data and the batch only, not on the iterate, so the batch
// matrices of all runs and of a range of t are built at once (k_mb_batches, one
// block per (run, t): the gather of s rows and s D^2 terms), and only the D x D
// recurrence runs in order (k_mb_iterate, one wave per run).  The range of t is
// sized so that the stored batch matrices stay within kMbBufBytes; the iterates
// carry over between ranges in a per-run state record.
#include "common.h"

namespace mapi {

constexpr int kMbThreads = 256;
constexpr int kMbMaxD = 64;
constexpr int kMbPairs = kMbMaxD * kMbMaxD / kMbThreads;   // 16
constexpr int kMbLdsFloats = 128 * kMbMaxD;                  // gathered samples' LDS buffer (32 KiB)
constexpr int kMbMaxChunk = 1024;                            // samples per gather pass at most
constexpr int kMbIdx = kMbMaxChunk / kMbThreads;             // sample indices per thread and pass
constexpr int kMbGather = kMbLdsFloats / kMbThreads;         // gathered floats per thread and pass
constexpr int kMbRun = 16;                                   // min1 terms per float32 run of a chain (narrow batches)
constexpr int kMbIterLds = 16384;                            // staged batch-matrix floats of the recurrence (64 KiB)
constexpr int kMbIterBatch = 16;                             // staging loads in flight per lane
constexpr size_t kMbBufBytes = size_t(256) << 20;           // stored batch matrices per range of t

// Iterate of one run between ranges of t.
struct MbState {
  float w[kMbMaxD], wp[kMbMaxD];
  double nu;
  int32_t it, status;
};

template <int OP>
__device__ __forceinline__ double mb_term(float a, float b) {
  if constexpr (OP == MAPI_OP_MIN1) {
    const float bb = fabsf(b);
    return (double)__builtin_amdgcn_fmed3f(flip_sign(a, sign_bit(b)), -bb, bb);   // exact in float32
  } else {
    return (double)a * (double)b;                                                  // exact in float64
  }
}

// Batch matrices of t = t0 .. t0 + nt - 1, into Abuf[(run * nt + t - t0) * D^2 + k D + l].
// With DD = D^2 < 256 pairs the block splits the samples into SL = 256 / DD slices:
// thread (slice, p) sums the terms of pair p over samples slice, slice + SL, ... of
// each gathered chunk (in four interleaved chains, added in a fixed order), and the
// slice partials are added in slice order.
// With DD >= 256 (WIDE) each thread sums up to kMbPairs pairs over all samples in order.
template <int OP, bool WIDE>
__global__ void __launch_bounds__(kMbThreads)
k_mb_batches(const float* __restrict__ X, int64_t N, int D, int64_t ldx, const int32_t* __restrict__ idx, int s,
             int T, int t0, int nt, float* __restrict__ Abuf, int32_t* __restrict__ bad_index) {
  __shared__ float xb[kMbLdsFloats];
  __shared__ int32_t jb[kMbMaxChunk];
  __shared__ double part[kMbThreads];
  const int tid = threadIdx.x;
  const int run = blockIdx.x / nt, tl = blockIdx.x - run * nt;
  const int DD = D * D;
  constexpr bool wide = WIDE;
  constexpr int GB = WIDE ? 8 : 16;   // gather loads in flight per thread (keeps the occupancy of the sums)
  constexpr int NQ = WIDE ? kMbPairs : 1;
  const int SL = wide ? 1 : kMbThreads / DD;
  const int slice = wide ? 0 : tid / DD;
  const bool active = wide || tid < SL * DD;
  const int32_t* B = idx + ((int64_t)run * T + t0 + tl) * s;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  // samples per gather: as many as the buffer holds (819 at D = 10), at most kMbMaxChunk
  const int chunk = min(kMbMaxChunk, kMbLdsFloats / D);
  for (int i0 = 0; i0 < s; i0 += chunk) {
    const int c = min(chunk, s - i0);
    __syncthreads();   // the previous chunk's readers are done
    // the chunk's sample indices first (an index outside [0, N) is reported after the
    // run and never used as an address), then the rows: each thread issues all of its
    // index loads (at most kMbIdx) before it checks the first, and its row loads in
    // passes of GB before it stores the first (at most kMbGather floats per chunk), so a
    // chunk costs one memory round trip for the indices and one or two for the rows
    int32_t jv[kMbIdx];
#pragma unroll
    for (int q = 0; q < kMbIdx; ++q) {
      const int i = tid + q * kMbThreads;
      jv[q] = i < c ? B[i0 + i] : 0;
    }
#pragma unroll
    for (int q = 0; q < kMbIdx; ++q) {
      const int i = tid + q * kMbThreads;
      if (i < c) {
        const int32_t j = jv[q];
        const bool ok = j >= 0 && (int64_t)j < N;
        if (!ok) atomicOr(bad_index, 1);
        jb[i] = ok ? j : 0;
      }
    }
    __syncthreads();
    // element e = tid + kMbThreads q of the chunk is coordinate k of sample i (e = i D + k),
    // advanced by kMbThreads = qd D + rd per step; i is clamped to the chunk, so every
    // address is that of a checked sample row
    {
      const int n_e = c * D, qd = kMbThreads / D, rd = kMbThreads - qd * D;
      int i = tid / D, k = tid - (tid / D) * D;
#pragma unroll 1
      for (int q0 = 0; q0 < kMbGather && tid + q0 * kMbThreads < n_e; q0 += GB) {
        float gv[GB];
#pragma unroll
        for (int q = 0; q < GB; ++q) {
          const int e = tid + (q0 + q) * kMbThreads;
          gv[q] = e < n_e ? X[(int64_t)jb[min(i, c - 1)] * ldx + k] : 0.0f;
          i += qd;
          k += rd;
          if (k >= D) {
            k -= D;
            ++i;
          }
        }
#pragma unroll
        for (int q = 0; q < GB; ++q) {
          const int e = tid + (q0 + q) * kMbThreads;
          if (e < n_e) xb[e] = gv[q];
        }
      }
    }
    __syncthreads();
    if (!active) continue;
    if constexpr (WIDE) {
      // samples outside, this thread's pairs inside: each pair still sums its samples in order
      int kq[NQ], lq[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int p = min(tid + q * kMbThreads, DD - 1);
        kq[q] = p / D;
        lq[q] = p - kq[q] * D;
      }
#pragma unroll 2
      for (int i = 0; i < c; ++i) {
        const float* xi = xb + i * D;
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] += mb_term<OP>(xi[kq[q]], xi[lq[q]]);
      }
    } else {
      // four independent float64 chains (samples slice + SL (4 m + r) into chain r), added
      // in a fixed order: the adds do not wait on each other
      const int p = tid - slice * DD;
      const int k = p / D, l = p - k * D;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int i = slice;
      if constexpr (OP == MAPI_OP_MIN1) {
        // min1 terms are exact in float32: each chain sums runs of kMbRun terms in float32
        // and adds the runs in float64
        float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f, f3 = 0.0f;
        int run_len = 0;
        for (; i + 3 * SL < c; i += 4 * SL) {
          f0 += (float)mb_term<OP>(xb[i * D + k], xb[i * D + l]);
          f1 += (float)mb_term<OP>(xb[(i + SL) * D + k], xb[(i + SL) * D + l]);
          f2 += (float)mb_term<OP>(xb[(i + 2 * SL) * D + k], xb[(i + 2 * SL) * D + l]);
          f3 += (float)mb_term<OP>(xb[(i + 3 * SL) * D + k], xb[(i + 3 * SL) * D + l]);
          if (++run_len == kMbRun) {
            a0 += f0;
            a1 += f1;
            a2 += f2;
            a3 += f3;
            f0 = f1 = f2 = f3 = 0.0f;
            run_len = 0;
          }
        }
        a0 += f0;
        a1 += f1;
        a2 += f2;
        a3 += f3;
      } else {
        for (; i + 3 * SL < c; i += 4 * SL) {
          a0 += mb_term<OP>(xb[i * D + k], xb[i * D + l]);
          a1 += mb_term<OP>(xb[(i + SL) * D + k], xb[(i + SL) * D + l]);
          a2 += mb_term<OP>(xb[(i + 2 * SL) * D + k], xb[(i + 2 * SL) * D + l]);
          a3 += mb_term<OP>(xb[(i + 3 * SL) * D + k], xb[(i + 3 * SL) * D + l]);
        }
      }
      for (; i < c; i += SL) a0 += mb_term<OP>(xb[i * D + k], xb[i * D + l]);
      acc[0] += (a0 + a1) + (a2 + a3);
    }
  }
  const double inv_s = 1.0 / (double)s;
  float* out = Abuf + ((int64_t)run * nt + tl) * DD;
  if constexpr (WIDE) {
    for (int q = 0; q < NQ; ++q) {
      const int p = tid + q * kMbThreads;
      if (p < DD) out[p] = (float)(acc[q] * inv_s);
    }
    return;
  }
  part[tid] = active ? acc[0] : 0.0;
  __syncthreads();
  if (tid < DD) {
    double sum = 0.0;
    for (int sl = 0; sl < SL; ++sl) sum += part[sl * DD + tid];
    out[tid] = (float)(sum * inv_s);
  }
}


// The recurrence over the stored batch matrices of one range of t; one wave per
// run, lane l < D holding w_l and w_{t-1, l}.  `first` starts from w0, `last`
// finishes (optional l2 step, output, run record); otherwise the iterate is kept
// in the run's state record.
template <int OP>
__global__ void __launch_bounds__(kWave)
k_mb_iterate(const float* __restrict__ Abuf, int D, int nt, float beta, MbState* __restrict__ states, int first,
             int last, const float* __restrict__ w0, float* __restrict__ w_out, int final_l2,
             MbRun* __restrict__ runs) {
  const int run = blockIdx.x, l = threadIdx.x;
  const bool mine = l < D;
  MbState* S = states + run;
  float w = 0.0f, wp = 0.0f;
  double nu = 0.0;
  int it = 0, status = MAPI_OK;
  if (first) {
    if (mine) w = w0[(int64_t)run * D + l];
  } else {
    if (mine) {
      w = S->w[l];
      wp = S->wp[l];
    }
    nu = S->nu;
    it = S->it;
    status = S->status;
  }
  // the run's batch matrices of this range are contiguous: they are copied into LDS a
  // stage of ns steps at a time with every load of a lane issued before its first store,
  // so the steps read A without a memory round trip each
  __shared__ __align__(16) float As[kMbIterLds];
  const int DD = D * D;
  const int ns = kMbIterLds / DD;   // >= 4: DD <= 4096
  for (int t0 = 0; t0 < nt && status == MAPI_OK; t0 += ns) {
    const int cnt = min(ns, nt - t0);
    const float* src = Abuf + ((int64_t)run * nt + t0) * DD;
    const int nf = cnt * DD;
    for (int e0 = 0; e0 < nf; e0 += kMbIterBatch * kWave) {
      float v[kMbIterBatch];
#pragma unroll
      for (int q = 0; q < kMbIterBatch; ++q) {
        const int e = e0 + q * kWave + l;
        v[q] = e < nf ? src[e] : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < kMbIterBatch; ++q) {
        const int e = e0 + q * kWave + l;
        if (e < nf) As[e] = v[q];
      }
    }
    __syncthreads();
    for (int tl = 0; tl < cnt; ++tl) {
      const float* A = As + tl * DD + l * D;
      float y = 0.0f;
      for (int m = 0; m < D; ++m) {
        const float wm = __shfl(w, m);
        if (mine) y = op_acc<OP>(y, A[m], wm, sign_bit(wm));
      }
      const float wn = mine ? fmaf(-beta, wp, y) : 0.0f;
      nu = wave_total_f64(mine ? fabs((double)wn) : 0.0);
      if (!(nu > 0.0) || !(nu < INFINITY)) {
        status = MAPI_ERR_DEGENERATE;
        break;
      }
      wp = (float)((double)w / nu);
      w = (float)((double)wn / nu);
      ++it;
    }
    __syncthreads();   // the stage is read before the next one overwrites it
  }
  if (!last) {
    if (mine) {
      S->w[l] = w;
      S->wp[l] = wp;
    }
    if (l == 0) {
      S->nu = nu;
      S->it = it;
      S->status = status;
    }
    return;
  }
  double scale = 1.0;
  if (final_l2 && status == MAPI_OK) {
    const double q2 = wave_total_f64(mine ? (double)w * (double)w : 0.0);
    if (!(q2 > 0.0) || !(q2 < INFINITY)) status = MAPI_ERR_DEGENERATE;
    else scale = 1.0 / sqrt(q2);
  }
  if (mine) w_out[(int64_t)run * D + l] = (scale == 1.0) ? w : (float)((double)w * scale);
  if (l == 0) {
    runs[run].iters = it;
    runs[run].status = status;
    runs[run].nu = nu;
  }
}

int minibatch_max_d() { return kMbMaxD; }

static size_t mb_align(size_t x) { return (x + 255) / 256 * 256; }

// Batches per range of t: as many as keep runs x range x D^2 stored floats within kMbBufBytes.
int minibatch_range(int D, int T, int runs) {
  const size_t per_t = (size_t)runs * (size_t)D * (size_t)D * sizeof(float);
  size_t r = kMbBufBytes / (per_t > 0 ? per_t : 1);
  if (r < 1) r = 1;
  if (r > (size_t)T) r = (size_t)T;
  return (int)(r < 1 ? 1 : r);
}

size_t minibatch_workspace_bytes(int D, int range, int runs) {
  const size_t buf = (size_t)runs * (size_t)(range < 1 ? 1 : range) * (size_t)D * (size_t)D * sizeof(float);
  return mb_align(buf) + (size_t)runs * sizeof(MbState);
}

hipError_t launch_minibatch(const float* X, int64_t N, int D, int64_t ldx, const int32_t* idx, int s, int T, float beta,
                            int op, int runs, const float* w0, float* w_out, int final_l2, MbRun* ri,
                            int32_t* bad_index, int range, void* ws, hipStream_t st) {
  if (op != MAPI_OP_MIN1 && op != MAPI_OP_DOT) return hipErrorInvalidValue;
  const int R = range < 1 ? 1 : range;
  float* Abuf = static_cast<float*>(ws);
  MbState* states = reinterpret_cast<MbState*>(static_cast<char*>(ws) +
                                               mb_align((size_t)runs * (size_t)R * D * D * sizeof(float)));
  if (T == 0) {
    if (op == MAPI_OP_MIN1)
      hipLaunchKernelGGL(k_mb_iterate<MAPI_OP_MIN1>, dim3(runs), dim3(kWave), 0, st, Abuf, D, 0, beta, states, 1, 1,
                         w0, w_out, final_l2, ri);
    else
      hipLaunchKernelGGL(k_mb_iterate<MAPI_OP_DOT>, dim3(runs), dim3(kWave), 0, st, Abuf, D, 0, beta, states, 1, 1, w0,
                         w_out, final_l2, ri);
    return hipGetLastError();
  }
  for (int t0 = 0; t0 < T; t0 += R) {
    const int nt = min(R, T - t0);
    const int first = t0 == 0, last = t0 + nt == T;
    const unsigned grid = (unsigned)((int64_t)runs * nt);
    if (op == MAPI_OP_MIN1) {
      if (D * D >= kMbThreads)
        hipLaunchKernelGGL((k_mb_batches<MAPI_OP_MIN1, true>), dim3(grid), dim3(kMbThreads), 0, st, X, N, D, ldx, idx,
                           s, T, t0, nt, Abuf, bad_index);
      else
        hipLaunchKernelGGL((k_mb_batches<MAPI_OP_MIN1, false>), dim3(grid), dim3(kMbThreads), 0, st, X, N, D, ldx, idx,
                           s, T, t0, nt, Abuf, bad_index);
      hipLaunchKernelGGL(k_mb_iterate<MAPI_OP_MIN1>, dim3(runs), dim3(kWave), 0, st, Abuf, D, nt, beta, states, first,
                         last, w0, w_out, final_l2, ri);
    } else {
      if (D * D >= kMbThreads)
        hipLaunchKernelGGL((k_mb_batches<MAPI_OP_DOT, true>), dim3(grid), dim3(kMbThreads), 0, st, X, N, D, ldx, idx, s,
                           T, t0, nt, Abuf, bad_index);
      else
        hipLaunchKernelGGL((k_mb_batches<MAPI_OP_DOT, false>), dim3(grid), dim3(kMbThreads), 0, st, X, N, D, ldx, idx,
                           s, T, t0, nt, Abuf, bad_index);
      hipLaunchKernelGGL(k_mb_iterate<MAPI_OP_DOT>, dim3(runs), dim3(kWave), 0, st, Abuf, D, nt, beta, states, first,
                         last, w0, w_out, final_l2, ri);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mapi
