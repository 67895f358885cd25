// Column-split PageRank product (eq. 11 split sums) for graphs whose iterate does not
// fit one XCD's L2.
//
// The in-link gathers w[j] of the plain CSR product hit the whole iterate at random
// (16 MiB at n = 2^22), so nearly every gather misses the 4 MiB L2 of its XCD and
// moves a whole cache sector for 4 useful bytes.  Here the sources are cut into K = 8
// column blocks of ceil(n / 8) nodes (2 MiB of float32 w at n = 2^22), and the CSR is
// re-laid out once per solve so that block k's entries of every row are contiguous.
// Workgroup b handles column block b % 8: with the round-robin dispatch of workgroups
// to the 8 XCDs, every XCD gathers from one block only, which stays in its L2.
// Each block yields a partial row sum per row; a combine kernel adds the K partials in
// block order (plus the teleport / dangling terms) and forms the normaliser's partials.
//
// Layout of the split matrix (device, built by launch_split_build):
//   len[k * n + i]   uint8   entries of row i in block k (< 255; a graph with a longer
//                            block row keeps the plain product)
//   base[k * nch + c] int32  offset of chunk c (64 rows) of block k in colS / valS
//   colS, valS       nnz     block 0's rows in order, then block 1's, ...; within a
//                            block row the entries keep their order in the input row
//   part[k * n + i]  T       block k's partial sum of row i (per product)
//
// Hub sources.  Out-degrees here are Zipf-distributed: a few thousand sources per
// block hold about half of its links, and the gathers of each such source land on one
// L2 line up to hundreds of thousands of times per product.  The kSplitHubSlots
// sources of each block with the most links (above a power-of-two threshold chosen per
// block) are therefore "hubs": every workgroup copies their iterate values into LDS
// once per product, and their links carry the LDS slot (stored as ~slot, a negative
// index) instead of the source, which takes about half of the gathers off the L2.
// Which sources are hubs and which slot each gets changes no value.
//   deg[j]           int32   estimated links with source j (1 / its link value, from a
//                            sample of the rows)
//   slot[j]          int32   LDS slot of hub j, -1 otherwise
//   hubs[k * H + s]  int32   source held in slot s of block k; nhub[k] slots in use
//   hval[k * H + s]  T       the iterate value of that source (gathered per product)
#include <algorithm>

#include "common.h"

namespace mapi {

constexpr int kSplitBlocks = 8;      // column blocks: one per XCD
constexpr int kSplitChunk = 64;      // rows per base entry (one wave, one lane per row)
constexpr int kSplitMaxLen = 255;    // block-row lengths fit uint8 below this
#ifndef MAPI_SPLIT_HUB_SLOTS
#define MAPI_SPLIT_HUB_SLOTS 3072
#endif
#ifndef MAPI_SPLIT_HUB_VALUES
#define MAPI_SPLIT_HUB_VALUES 1
#endif
constexpr int kSplitHubSlots = MAPI_SPLIT_HUB_SLOTS;   // hub sources per block held in LDS
constexpr int kSplitHubMinDeg = 32;  // no hub below this many links
// Hub values gathered once per product into a slot-ordered array, so that every
// workgroup fills its LDS copy with contiguous reads (otherwise each workgroup gathers
// them from the iterate itself)
constexpr bool kSplitHubValues = MAPI_SPLIT_HUB_VALUES != 0;

int64_t split_block_cols(int64_t n) { return (n + kSplitBlocks - 1) / kSplitBlocks; }
int64_t split_chunks(int64_t n) { return (n + kSplitChunk - 1) / kSplitChunk; }

// j / bcols for 0 <= j < 2^31 without a 64-bit division: a float estimate corrected by
// one step either way (the estimate is within one of the quotient).
__device__ __forceinline__ int block_of(int32_t j, int32_t bcols, float inv_bcols) {
  int k = (int)((float)j * inv_bcols);
  if (k * bcols > j) --k;
  else if ((k + 1) * bcols <= j) ++k;
  return k;
}

// Hub ranking of a link: a column-stochastic link value of a graph is 1 / out-degree of
// its source, so its reciprocal estimates that count.
__device__ __forceinline__ int32_t degree_estimate(float h) {
  return (h > 0.0f && h <= 1.0f) ? (int32_t)fminf(1.0f / h + 0.5f, 1.0e9f) : 1;
}

// Exclusive prefix sum over the 64 lanes of a wave (int).
__device__ __forceinline__ int wave_excl_scan(int v) {
  const int lane = threadIdx.x & (kWave - 1);
  int x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  return x - v;
}

// Count each row's entries per column block (one lane per row, one wave per chunk of 64
// rows) and each chunk's total per block.  flags bit 0: some block row has kSplitMaxLen
// or more entries (the split layout is not used); the CSR was validated before.
__global__ void __launch_bounds__(256)
k_split_count(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col, const float* __restrict__ val,
              int64_t n, int64_t bcols, uint8_t* __restrict__ len, int32_t* __restrict__ csum, int64_t nch,
              int32_t* __restrict__ flags, int32_t* __restrict__ deg) {
  const int lane = threadIdx.x & (kWave - 1);
  const float inv_bcols = 1.0f / (float)bcols;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; c < nch; c += waves) {
    const int64_t i = c * kSplitChunk + lane;
    int cnt[kSplitBlocks];
#pragma unroll
    for (int k = 0; k < kSplitBlocks; ++k) cnt[k] = 0;
    if (i < n) {
      const int32_t p1 = row_ptr[i + 1];
      // hub ranking from the link values (no atomic per link: the busiest sources have
      // millions); rows i = 0 mod 8 suffice to see every source with more than a few
      // dozen links, and any estimate is valid -- a hub only moves where its value is read
      const bool sample = (i & 7) == 0;
      for (int32_t p = row_ptr[i]; p < p1; ++p) {
        const int32_t j = col[p];
        const int kb = block_of(j, (int32_t)bcols, inv_bcols);
#pragma unroll
        for (int k = 0; k < kSplitBlocks; ++k) cnt[k] += (kb == k) ? 1 : 0;
        if (sample) deg[j] = degree_estimate(val[p]);
      }
    }
    bool over = false;
#pragma unroll
    for (int k = 0; k < kSplitBlocks; ++k) {
      over |= cnt[k] >= kSplitMaxLen;
      if (i < n) len[k * n + i] = (uint8_t)(cnt[k] < kSplitMaxLen ? cnt[k] : kSplitMaxLen);
      int s = cnt[k];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, kWave);
      if (lane == 0) csum[k * nch + c] = s;
    }
    if (over) atomicOr(flags, 1);
  }
}

// Exclusive scan of the chunk totals of every block in block order, in place, so that
// they become absolute positions in colS / valS: tiles of 1024 totals (256 threads, four
// consecutive totals each) are summed, the tile sums scanned by one block, and each tile
// rescanned from its offset.  Integer sums, so the order does not matter.
constexpr int kScanTile = 1024;

__device__ __forceinline__ int block_excl_scan_256(int v, int* sh, int* total) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int ex = wave_excl_scan(v);
  if (lane == kWave - 1) sh[wave] = ex + v;
  __syncthreads();
  int off = 0, tot = 0;
  for (int q = 0; q < 4; ++q) {
    if (q < wave) off += sh[q];
    tot += sh[q];
  }
  __syncthreads();
  *total = tot;
  return off + ex;
}

__global__ void __launch_bounds__(256) k_scan_tile_sums(const int32_t* __restrict__ v, int64_t total,
                                                        int32_t* __restrict__ tsum) {
  __shared__ int sh[4];
  int s = 0;
  for (int q = 0; q < 4; ++q) {
    const int64_t i = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 4 + q;
    s += i < total ? v[i] : 0;
  }
  int tot;
  (void)block_excl_scan_256(s, sh, &tot);
  if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256) k_scan_tile_offsets(int32_t* __restrict__ tsum, int ntiles) {
  __shared__ int sh[4];
  int carry = 0;
  for (int t0 = 0; t0 < ntiles; t0 += 256) {
    const int t = t0 + threadIdx.x;
    const int v = t < ntiles ? tsum[t] : 0;
    int tot;
    const int ex = block_excl_scan_256(v, sh, &tot);
    if (t < ntiles) tsum[t] = carry + ex;
    carry += tot;
  }
}

__global__ void __launch_bounds__(256) k_scan_tile_apply(int32_t* __restrict__ v, int64_t total,
                                                         const int32_t* __restrict__ toff) {
  __shared__ int sh[4];
  int x[4], s = 0;
  for (int q = 0; q < 4; ++q) {
    const int64_t i = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 4 + q;
    x[q] = i < total ? v[i] : 0;
    s += x[q];
  }
  int tot;
  int run = toff[blockIdx.x] + block_excl_scan_256(s, sh, &tot);
  for (int q = 0; q < 4; ++q) {
    const int64_t i = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 4 + q;
    if (i < total) v[i] = run;
    run += x[q];
  }
}

// Per block, a histogram of floor(log2(degree)) of its sources (32 bins).
__global__ void __launch_bounds__(256)
k_split_hub_hist(const int32_t* __restrict__ deg, int64_t n, int64_t bcols, int32_t* __restrict__ hist) {
  __shared__ int32_t lh[kSplitBlocks * 32];
  const float inv_bcols = 1.0f / (float)bcols;
  for (int q = threadIdx.x; q < kSplitBlocks * 32; q += blockDim.x) lh[q] = 0;
  __syncthreads();
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const int d = deg[j];
    if (d >= kSplitHubMinDeg) atomicAdd(&lh[block_of((int32_t)j, (int32_t)bcols, inv_bcols) * 32 + (31 - __clz(d))], 1);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kSplitBlocks * 32; q += blockDim.x)
    if (lh[q]) atomicAdd(&hist[q], lh[q]);
}

// Per block, the smallest power-of-two degree threshold (at least kSplitHubMinDeg) above
// which at most kSplitHubSlots sources lie; the sources at or above it are the hubs.
__global__ void k_split_hub_threshold(const int32_t* __restrict__ hist, int32_t* __restrict__ thr,
                                      int32_t* __restrict__ nhub) {
  const int k = threadIdx.x;
  if (k >= kSplitBlocks) return;
  int cum = 0, b = 31;
  for (; b >= 0; --b) {
    if (cum + hist[k * 32 + b] > kSplitHubSlots) break;
    cum += hist[k * 32 + b];
  }
  const int t = b + 1;    // bins t..31 fit the slots
  thr[k] = t >= 31 ? INT32_MAX : max(kSplitHubMinDeg, 1 << t);
  nhub[k] = 0;
}

// Slots of the hubs (any order: a slot only places a value in LDS).  Atomics on the
// eight counters, which share a cache line, are serialised by the device, so each pass
// of a workgroup over kHubPass sources counts its hubs per block in LDS and takes its
// slots with one global atomic per block it touched (one per wave cost 0.3 ms with
// about 24 000 hubs).
constexpr int kHubPass = 16;       // sources per thread and pass
__global__ void __launch_bounds__(256)
k_split_hub_assign(const int32_t* __restrict__ deg, int64_t n, int64_t bcols, const int32_t* __restrict__ thr,
                   int32_t* __restrict__ nhub, int32_t* __restrict__ slot, int32_t* __restrict__ hubs) {
  __shared__ int cnt[kSplitBlocks], base[kSplitBlocks];
  const float inv_bcols = 1.0f / (float)bcols;
  const int64_t span = (int64_t)blockDim.x * kHubPass;
  for (int64_t jb = (int64_t)blockIdx.x * span; jb < n; jb += (int64_t)gridDim.x * span) {
    if (threadIdx.x < kSplitBlocks) cnt[threadIdx.x] = 0;
    __syncthreads();
    int kq[kHubPass], lo[kHubPass];
#pragma unroll
    for (int p = 0; p < kHubPass; ++p) {
      const int64_t j = jb + (int64_t)p * blockDim.x + threadIdx.x;
      kq[p] = -1;
      lo[p] = 0;
      if (j < n) {
        const int k = block_of((int32_t)j, (int32_t)bcols, inv_bcols);
        if (deg[j] >= thr[k]) {
          kq[p] = k;
          lo[p] = atomicAdd(&cnt[k], 1);
        }
      }
    }
    __syncthreads();
    if (threadIdx.x < kSplitBlocks) base[threadIdx.x] = cnt[threadIdx.x] ? atomicAdd(&nhub[threadIdx.x], cnt[threadIdx.x]) : 0;
    __syncthreads();
#pragma unroll
    for (int p = 0; p < kHubPass; ++p) {
      const int64_t j = jb + (int64_t)p * blockDim.x + threadIdx.x;
      if (j >= n) continue;
      int32_t s = kq[p] >= 0 ? base[kq[p]] + lo[p] : -1;
      if (s >= kSplitHubSlots) s = -1;    // cannot happen: the threshold admits at most kSplitHubSlots
      if (s >= 0) hubs[kq[p] * kSplitHubSlots + s] = (int32_t)j;
      slot[j] = s;
    }
    __syncthreads();   // base and cnt are rewritten by the next pass
  }
}

// Scatter every entry to its block's run: lane = row, block rows start at the chunk's
// offset plus the wave's exclusive scan of the block-row lengths.  A chunk's entries of
// one block form one contiguous range of colS / valS, so a wave assembles its chunk in
// LDS (its eight ranges back to back) and then writes each range with coalesced stores;
// a chunk with more than kScatterCap links writes its entries one by one.
constexpr int kScatterCap = 1536;    // links of a chunk assembled in LDS (per wave)
__global__ void __launch_bounds__(256)
k_split_scatter(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col, const float* __restrict__ val,
                int64_t n, int64_t bcols, const uint8_t* __restrict__ len, const int32_t* __restrict__ base,
                int64_t nch, const int32_t* __restrict__ slot, const int32_t* __restrict__ thr,
                int32_t* __restrict__ colS, float* __restrict__ valS) {
  __shared__ int32_t lc[256 / kWave][kScatterCap];
  __shared__ float lv[256 / kWave][kScatterCap];
  const float inv_bcols = 1.0f / (float)bcols;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; c < nch; c += waves) {
    const int64_t i = c * kSplitChunk + lane;
    int pos[kSplitBlocks], start[kSplitBlocks];
    int tot = 0;                                 // the chunk's links (the same in every lane)
#pragma unroll
    for (int k = 0; k < kSplitBlocks; ++k) {
      const int l = i < n ? (int)len[k * n + i] : 0;
      const int ex = wave_excl_scan(l);
      start[k] = tot;
      pos[k] = ex;
      tot += __builtin_amdgcn_readfirstlane(__shfl(ex + l, kWave - 1, kWave));
    }
    const bool staged = tot <= kScatterCap;
#pragma unroll
    for (int k = 0; k < kSplitBlocks; ++k) pos[k] += staged ? start[k] : base[k * nch + c];
    // the lane's links: destination, stored source (~slot for a hub) and value.  Only a
    // link whose own value ranks its source as a hub looks up the slot (a few thousand
    // sources: the lookups stay in cache); a source without a slot is gathered from memory
    auto link = [&](int32_t p, int* dst, int32_t* cv, float* hv) {
      const int32_t j = col[p];
      const int kb = block_of(j, (int32_t)bcols, inv_bcols);
      int d = 0;
#pragma unroll
      for (int k = 0; k < kSplitBlocks; ++k) {
        if (kb == k) {
          d = pos[k];
          pos[k] += 1;
        }
      }
      const float h = val[p];
      const int32_t hs = degree_estimate(h) >= thr[kb] ? slot[j] : -1;
      *dst = d;
      *cv = hs >= 0 ? ~hs : j;
      *hv = h;
    };
    if (i < n) {
      const int32_t p0 = row_ptr[i], p1 = row_ptr[i + 1];
      int d;
      int32_t cv;
      float hv;
      if (staged) {
        for (int32_t p = p0; p < p1; ++p) {
          link(p, &d, &cv, &hv);
          lc[wv][d] = cv;
          lv[wv][d] = hv;
        }
      } else {
        for (int32_t p = p0; p < p1; ++p) {
          link(p, &d, &cv, &hv);
          colS[d] = cv;
          valS[d] = hv;
        }
      }
    }
    if (staged) {
      // the wave's LDS writes before its reads of other lanes' entries
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int k = 0; k < kSplitBlocks; ++k) {
        const int kt = (k + 1 < kSplitBlocks ? start[k + 1] : tot) - start[k];
        const int64_t b0 = base[k * nch + c];
        for (int e = lane; e < kt; e += kWave) {
          colS[b0 + e] = lc[wv][start[k] + e];
          valS[b0 + e] = lv[wv][start[k] + e];
        }
      }
      // every lane's LDS reads before the next chunk's writes
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
}

// Block k's partial sum of every row: workgroup b takes block b % K; its waves take
// groups of kSplitBatch consecutive chunks of 64 rows, lane l row c * 64 + l of each.
// A chunk's links of one block are contiguous in colS / valS (about 115 here), so the
// wave first copies them into its LDS with coalesced loads -- every byte crosses HBM
// once -- and each lane then reads its row's links from LDS and gathers w.  A row's
// links of one block are few (about two), so the lane issues the gathers of its first
// kSplitFirst links together.  Working on kSplitBatch chunks at once keeps more loads in
// flight per wave.  A chunk with more than kSplitCap links is read from HBM lane by
// lane instead.  Each row's terms are added in link order, as in the plain product
// (k_csr.hip).
#ifndef MAPI_SPLIT_BATCH
#define MAPI_SPLIT_BATCH 2
#endif
#ifndef MAPI_SPLIT_FIRST
#define MAPI_SPLIT_FIRST 4
#endif
constexpr int kSplitBatch = MAPI_SPLIT_BATCH;
constexpr int kSplitFirst = MAPI_SPLIT_FIRST;
constexpr int kSplitCap = 192;        // links of one chunk staged in LDS
constexpr int kSplitWaves = 4;        // waves per workgroup

template <int METHOD, typename T>
__device__ __forceinline__ T split_term(T acc, float h, T wj, float af, float cf, double ad, double cd) {
  if constexpr (METHOD == MAPI_METHOD_MAPI) {
    if constexpr (sizeof(T) == 4) {
      const float g = fmaf(af, h, cf);
      return acc + (__builtin_amdgcn_fmed3f(wj, -g, g) - __builtin_amdgcn_fmed3f(wj, -cf, cf));
    } else {
      const double g = ad * (double)h + cd;
      return acc + (fmin(fmax(wj, -g), g) - fmin(fmax(wj, -cd), cd));
    }
  } else {
    return fma((T)h, wj, acc);
  }
}

// The iterate values of block k's hubs in slot order (one gather per hub and product).
template <typename T>
__global__ void __launch_bounds__(256)
k_split_hub_values(const T* __restrict__ w, int64_t n, const int32_t* __restrict__ hubs,
                   const int32_t* __restrict__ nhub, T* __restrict__ hval, const SolveState* __restrict__ st) {
  if (state_done(st)) return;
  const int k = blockIdx.y;
  const int nh = min(nhub[k], kSplitHubSlots);
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nh; q += gridDim.x * blockDim.x) {
    int32_t j = hubs[k * kSplitHubSlots + q];
    if (!MAPI_DCHECK(st, j >= 0 && (int64_t)j < n, 3)) j = 0;   // a hub outside 0..n-1
    hval[k * kSplitHubSlots + q] = w[j];
  }
}

template <int METHOD, typename T>
__global__ void __launch_bounds__(kSplitWaves * kWave)
k_csr_split_product(const uint8_t* __restrict__ len, const int32_t* __restrict__ base, const int32_t* __restrict__ colS,
                    const float* __restrict__ valS, int64_t n, int64_t nch, const T* __restrict__ w,
                    const int32_t* __restrict__ hubs, const int32_t* __restrict__ nhub, const T* __restrict__ hval,
                    T* __restrict__ part, const SolveState* __restrict__ st, double alpha, double c) {
  constexpr int R = kSplitBatch, E = kSplitFirst, CAP = kSplitCap;
  constexpr int SWEEPS = CAP / kWave;
  __shared__ int32_t lcol[kSplitWaves][R][CAP];
  __shared__ float lval[kSplitWaves][R][CAP];
  __shared__ T lhub[kSplitHubSlots > 0 ? kSplitHubSlots : 1];
  if (state_done(st)) return;
  const int k = blockIdx.x % kSplitBlocks;
  if constexpr (kSplitHubSlots > 0) {
    const int nh = min(nhub[k], kSplitHubSlots);
    if constexpr (kSplitHubValues) {
      for (int q = threadIdx.x; q < nh; q += blockDim.x) lhub[q] = hval[k * kSplitHubSlots + q];
    } else {
      for (int q = threadIdx.x; q < nh; q += blockDim.x) lhub[q] = w[hubs[k * kSplitHubSlots + q]];
    }
    __syncthreads();
  }
  // w of a link's source: a hub's from LDS (stored as ~slot), any other's from memory.
  // Each read goes through a pointer of its own address space: merged into one read
  // through a generic pointer (a flat load), every gather would also wait on the LDS
  // counter and every hub read on the vector-memory counter.
  typedef __attribute__((address_space(1))) const T gmem_t;
  typedef __attribute__((address_space(3))) const T lmem_t;
  gmem_t* wg = (gmem_t*)w;
  lmem_t* wl = (lmem_t*)lhub;
  const int nh_k = kSplitHubSlots > 0 ? min(nhub[k], kSplitHubSlots) : 0;
  auto wsrc = [&](int32_t jj) -> T {
    T v;
    if (jj >= 0) {
      if (!MAPI_DCHECK(st, (int64_t)jj < n, 3)) jj = 0;        // a source outside 0..n-1
      v = wg[jj];
    } else {
      int32_t slot = ~jj;
      if (!MAPI_DCHECK(st, slot < nh_k, 3)) slot = 0;          // a hub slot not staged in LDS
      v = wl[slot];
    }
    return v;
  };
  const int64_t groups = gridDim.x / kSplitBlocks;
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const double ad = sizeof(T) == 4 ? (double)(float)alpha : alpha;
  const double cd = sizeof(T) == 4 ? (double)(float)c : c;
  const float af = (float)ad, cf = (float)cd;
  const uint8_t* lenk = len + (int64_t)k * n;
  const int32_t* basek = base + (int64_t)k * nch;
  T* partk = part + (int64_t)k * n;
  const int64_t wid = (int64_t)(blockIdx.x / kSplitBlocks) * kSplitWaves + wv;
  const int64_t nwaves = groups * kSplitWaves;
  for (int64_t c0 = wid * R; c0 < nch; c0 += nwaves * R) {
    int l[R], off[R], tot[R];
    int32_t b0[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = (c0 + r) * kSplitChunk + lane;
      l[r] = (c0 + r < nch && i < n) ? (int)lenk[i] : 0;
      b0[r] = c0 + r < nch ? basek[c0 + r] : 0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      off[r] = wave_excl_scan(l[r]);
      // the chunk's link count, the same in every lane: a wave-uniform value, so that the
      // staged and the unstaged reads below are separate branches, each through its own
      // address space (not one flat load of either)
      tot[r] = __builtin_amdgcn_readfirstlane(__shfl(off[r] + l[r], kWave - 1, kWave));
    }
    // the chunks' links into LDS: coalesced, every load of all R chunks issued first
    int32_t sc[R][SWEEPS];
    float sv[R][SWEEPS];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int q = 0; q < SWEEPS; ++q) {
        const int e = q * kWave + lane;
        sc[r][q] = 0;
        sv[r][q] = 0.0f;
        if (tot[r] <= CAP && e < tot[r]) {
          sc[r][q] = __builtin_nontemporal_load(colS + b0[r] + e);
          sv[r][q] = __builtin_nontemporal_load(valS + b0[r] + e);
        }
      }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int q = 0; q < SWEEPS; ++q) {
        const int e = q * kWave + lane;
        if (tot[r] <= CAP && e < tot[r]) {
          lcol[wv][r][e] = sc[r][q];
          lval[wv][r][e] = sv[r][q];
        }
      }
    // the wave's LDS writes before its reads of other lanes' entries
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // first E links of every row: indices and values, then all gathers, then the terms
    int32_t j[R][E];
    float h[R][E];
    T wj[R][E];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (tot[r] <= CAP) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          j[r][e] = e < l[r] ? lcol[wv][r][off[r] + e] : 0;
          h[r][e] = e < l[r] ? lval[wv][r][off[r] + e] : 0.0f;
        }
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          j[r][e] = e < l[r] ? __builtin_nontemporal_load(colS + b0[r] + off[r] + e) : 0;
          h[r][e] = e < l[r] ? __builtin_nontemporal_load(valS + b0[r] + off[r] + e) : 0.0f;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int e = 0; e < E; ++e) wj[r][e] = e < l[r] ? wsrc(j[r][e]) : T(0);
    T acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      acc[r] = T(0);
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (e < l[r]) acc[r] = split_term<METHOD, T>(acc[r], h[r][e], wj[r][e], af, cf, ad, cd);
    }
    // links past the first E of a row, one at a time
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (tot[r] <= CAP) {
        for (int e = E; e < l[r]; ++e)
          acc[r] = split_term<METHOD, T>(acc[r], lval[wv][r][off[r] + e], wsrc(lcol[wv][r][off[r] + e]), af, cf, ad, cd);
      } else {
        for (int e = E; e < l[r]; ++e) {
          const int32_t jj = __builtin_nontemporal_load(colS + b0[r] + off[r] + e);
          const float hh = __builtin_nontemporal_load(valS + b0[r] + off[r] + e);
          acc[r] = split_term<METHOD, T>(acc[r], hh, wsrc(jj), af, cf, ad, cd);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = (c0 + r) * kSplitChunk + lane;
      if (c0 + r < nch && i < n) partk[i] = acc[r];
    }
    // every lane's LDS reads of this group before the next group's writes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// y_i = scalars + (sum of the K partials in block order), as the plain product forms it
// from its row sum; one partial of sum |y_i| per workgroup for the normaliser.
template <int METHOD, typename T>
__global__ void __launch_bounds__(256)
k_csr_split_combine(const T* __restrict__ part, int64_t n, T* __restrict__ y, double* __restrict__ nparts,
                    const SolveState* __restrict__ st, double alpha, double c, double inv_n) {
  __shared__ double sh[16];
  if (state_done(st)) return;
  const double ad = sizeof(T) == 4 ? (double)(float)alpha : alpha;
  const double cd = sizeof(T) == 4 ? (double)(float)c : c;
  const double sbase = (METHOD == MAPI_METHOD_MAPI) ? st->ex[0] + st->ex[1] : (ad * inv_n) * st->ex[1] + cd * st->ex[0];
  double nrm = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    T a = T(0);
#pragma unroll
    for (int k = 0; k < kSplitBlocks; ++k) a += __builtin_nontemporal_load(part + (int64_t)k * n + i);
    const T yi = (METHOD == MAPI_METHOD_MAPI) ? (T)(sbase + (double)a) : (T)(ad * (double)a + sbase);
    y[i] = yi;
    nrm += fabs((double)yi);
  }
  const double bsum = block_sum_f64(nrm, sh);
  if (threadIdx.x == 0) nparts[blockIdx.x] = bsum;
}

static int split_grid(int64_t work, int per_block, int cap) {
  int64_t b = (work + per_block - 1) / per_block;
  if (b > cap) b = cap;
  return (int)(b < 1 ? 1 : b);
}

size_t split_csr_bytes(int64_t n, int64_t nnz, size_t es) {
  const int64_t nch = split_chunks(n);
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  return al((size_t)kSplitBlocks * n) + al(sizeof(int32_t) * kSplitBlocks * nch) + al(sizeof(int32_t) * nnz) +
         al(sizeof(float) * nnz) + al(es * kSplitBlocks * n) + al(sizeof(int32_t)) + 2 * al(sizeof(int32_t) * n) +
         al(sizeof(int32_t) * kSplitBlocks * (kSplitHubSlots + 34)) + al(es * kSplitBlocks * kSplitHubSlots) +
         al(sizeof(int32_t) * ((kSplitBlocks * nch + kScanTile - 1) / kScanTile));
}

SplitCsr split_csr_place(void* ws, int64_t n, int64_t nnz, size_t es) {
  const int64_t nch = split_chunks(n);
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  char* p = static_cast<char*>(ws);
  SplitCsr s;
  s.n = n;
  s.nnz = nnz;
  s.nch = nch;
  s.len = reinterpret_cast<uint8_t*>(p);
  p += al((size_t)kSplitBlocks * n);
  s.base = reinterpret_cast<int32_t*>(p);
  p += al(sizeof(int32_t) * kSplitBlocks * nch);
  s.col = reinterpret_cast<int32_t*>(p);
  p += al(sizeof(int32_t) * nnz);
  s.val = reinterpret_cast<float*>(p);
  p += al(sizeof(float) * nnz);
  s.part = p;
  p += al(es * kSplitBlocks * n);
  s.flags = reinterpret_cast<int32_t*>(p);
  p += al(sizeof(int32_t));
  s.deg = reinterpret_cast<int32_t*>(p);
  p += al(sizeof(int32_t) * n);
  s.slot = reinterpret_cast<int32_t*>(p);
  p += al(sizeof(int32_t) * n);
  s.hubs = reinterpret_cast<int32_t*>(p);          // kSplitBlocks * slots, then 8 counts,
  s.nhub = s.hubs + kSplitBlocks * kSplitHubSlots;  // 8 thresholds and 8 x 32 histogram bins
  s.thr = s.nhub + kSplitBlocks;
  s.hist = s.thr + kSplitBlocks;
  p += al(sizeof(int32_t) * kSplitBlocks * (kSplitHubSlots + 34));
  s.hval = p;
  p += al(es * kSplitBlocks * kSplitHubSlots);
  s.tsum = reinterpret_cast<int32_t*>(p);
  return s;
}

__global__ void k_split_fill_i32(int32_t* __restrict__ p, int64_t count, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_split_zero(int32_t* __restrict__ p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

hipError_t launch_split_count(const int32_t* row_ptr, const int32_t* col, const float* val, const SplitCsr& s,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_split_zero, dim3(split_grid(s.n, 256, 4096)), dim3(256), 0, st, s.deg, s.n);
  hipLaunchKernelGGL(k_split_zero, dim3(1), dim3(256), 0, st, s.hist, (int64_t)kSplitBlocks * 32);
  hipLaunchKernelGGL(k_split_count, dim3(split_grid(s.nch, 4, 16384)), dim3(256), 0, st, row_ptr, col, val, s.n,
                     split_block_cols(s.n), s.len, s.base, s.nch, s.flags, s.deg);
  return hipGetLastError();
}

hipError_t launch_split_fill(const int32_t* row_ptr, const int32_t* col, const float* val, const SplitCsr& s,
                             hipStream_t st) {
  const int64_t total = (int64_t)kSplitBlocks * s.nch;
  const int ntiles = (int)((total + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(k_scan_tile_sums, dim3(ntiles), dim3(256), 0, st, s.base, total, s.tsum);
  hipLaunchKernelGGL(k_scan_tile_offsets, dim3(1), dim3(256), 0, st, s.tsum, ntiles);
  hipLaunchKernelGGL(k_scan_tile_apply, dim3(ntiles), dim3(256), 0, st, s.base, total, s.tsum);
  const int64_t bcols = split_block_cols(s.n);
  const int ng = split_grid(s.n, 256, 4096);
  if (kSplitHubSlots > 0) {
    hipLaunchKernelGGL(k_split_hub_hist, dim3(ng), dim3(256), 0, st, s.deg, s.n, bcols, s.hist);
    hipLaunchKernelGGL(k_split_hub_threshold, dim3(1), dim3(64), 0, st, s.hist, s.thr, s.nhub);
  } else {
    hipLaunchKernelGGL(k_split_zero, dim3(1), dim3(64), 0, st, s.nhub, (int64_t)kSplitBlocks);
    hipLaunchKernelGGL(k_split_fill_i32, dim3(1), dim3(64), 0, st, s.thr, (int64_t)kSplitBlocks, INT32_MAX);
  }
  hipLaunchKernelGGL(k_split_hub_assign, dim3(split_grid(s.n, 256 * kHubPass, 1024)), dim3(256), 0, st, s.deg, s.n,
                     bcols, s.thr, s.nhub, s.slot, s.hubs);
  hipLaunchKernelGGL(k_split_scatter, dim3(split_grid(s.nch, 4, 16384)), dim3(256), 0, st, row_ptr, col, val, s.n,
                     bcols, s.len, s.base, s.nch, s.slot, s.thr, s.col, s.val);
  return hipGetLastError();
}

int split_combine_blocks(int64_t n) { return split_grid(n, 1024, 2048); }

// Workgroups per column block of the product: as many as the device keeps resident at
// once (its occupancy: registers and LDS, with the hub copy), so that none runs in a
// second round and fills its hub copy again.  The result does not depend on it.
template <int METHOD, typename T>
static int split_product_groups() {
  // computed once per instance, on the first call's device (thread-safe initialisation)
  static const int g = [] {
    int dev = 0, cus = 256, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_csr_split_product<METHOD, T>, kSplitWaves * kWave,
                                                     0) != hipSuccess || per_cu < 1)
      per_cu = 4;
    return std::max(1, per_cu * cus / kSplitBlocks);
  }();
  return g;
}

template <typename T>
hipError_t launch_csr_split_product(int method, const SplitCsr& s, const T* w, T* y, double* nparts, SolveState* st,
                                    double alpha, double c, double inv_n, hipStream_t stream) {
  // workgroups persistent over the chunks, as many per column block as stay resident
  const int groups = split_grid(s.nch, 4, method == MAPI_METHOD_MAPI ? split_product_groups<MAPI_METHOD_MAPI, T>()
                                                                     : split_product_groups<MAPI_METHOD_RPI, T>());
  const dim3 grid((unsigned)(groups * kSplitBlocks));
  T* part = static_cast<T*>(s.part);
  T* hval = static_cast<T*>(s.hval);
  if (kSplitHubValues && kSplitHubSlots > 0)
    hipLaunchKernelGGL(k_split_hub_values<T>, dim3((kSplitHubSlots + 255) / 256, kSplitBlocks), dim3(256), 0, stream, w,
                       s.n, s.hubs, s.nhub, hval, st);
  if (method == MAPI_METHOD_MAPI) {
    hipLaunchKernelGGL((k_csr_split_product<MAPI_METHOD_MAPI, T>), grid, dim3(kSplitWaves * kWave), 0, stream, s.len,
                       s.base, s.col, s.val, s.n, s.nch, w, s.hubs, s.nhub, hval, part, st, alpha, c);
    hipLaunchKernelGGL((k_csr_split_combine<MAPI_METHOD_MAPI, T>), dim3(split_combine_blocks(s.n)), dim3(256), 0,
                       stream, part, s.n, y, nparts, st, alpha, c, inv_n);
  } else {
    hipLaunchKernelGGL((k_csr_split_product<MAPI_METHOD_RPI, T>), grid, dim3(kSplitWaves * kWave), 0, stream, s.len,
                       s.base, s.col, s.val, s.n, s.nch, w, s.hubs, s.nhub, hval, part, st, alpha, c);
    hipLaunchKernelGGL((k_csr_split_combine<MAPI_METHOD_RPI, T>), dim3(split_combine_blocks(s.n)), dim3(256), 0,
                       stream, part, s.n, y, nparts, st, alpha, c, inv_n);
  }
  return hipGetLastError();
}
template hipError_t launch_csr_split_product<float>(int, const SplitCsr&, const float*, float*, double*, SolveState*,
                                                    double, double, double, hipStream_t);
template hipError_t launch_csr_split_product<double>(int, const SplitCsr&, const double*, double*, double*,
                                                     SolveState*, double, double, double, hipStream_t);

}  // namespace mapi
