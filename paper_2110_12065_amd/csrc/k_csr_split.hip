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
#include "common.h"

namespace mapi {

constexpr int kSplitBlocks = 8;      // column blocks: one per XCD
constexpr int kSplitChunk = 64;      // rows per base entry (one wave, one lane per row)
constexpr int kSplitMaxLen = 255;    // block-row lengths fit uint8 below this

int64_t split_block_cols(int64_t n) { return (n + kSplitBlocks - 1) / kSplitBlocks; }
int64_t split_chunks(int64_t n) { return (n + kSplitChunk - 1) / kSplitChunk; }

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
k_split_count(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col, int64_t n, int64_t bcols,
              uint8_t* __restrict__ len, int32_t* __restrict__ csum, int64_t nch, int32_t* __restrict__ flags) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; c < nch; c += waves) {
    const int64_t i = c * kSplitChunk + lane;
    int cnt[kSplitBlocks];
#pragma unroll
    for (int k = 0; k < kSplitBlocks; ++k) cnt[k] = 0;
    if (i < n) {
      const int32_t p1 = row_ptr[i + 1];
      for (int32_t p = row_ptr[i]; p < p1; ++p) {
        const int kb = (int)((int64_t)col[p] / bcols);
#pragma unroll
        for (int k = 0; k < kSplitBlocks; ++k) cnt[k] += (kb == k) ? 1 : 0;
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

// Exclusive scan of the chunk totals of every block in block order, in place, by one
// block of 1024 threads: thread t sums a contiguous segment of the totals, the segment
// sums are scanned across the block, then each thread rewrites its segment with running
// offsets -- absolute positions in colS / valS.
__global__ void __launch_bounds__(1024) k_split_scan(int32_t* __restrict__ csum, int64_t total) {
  __shared__ int64_t sh[16];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int64_t seg = (total + blockDim.x - 1) / blockDim.x;
  const int64_t b = (int64_t)threadIdx.x * seg, e = b + seg < total ? b + seg : total;
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += csum[i];
  // exclusive scan of the segment sums: within the wave, then across waves
  int64_t x = s;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int64_t y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  if (lane == kWave - 1) sh[wave] = x;
  __syncthreads();
  int64_t run = x - s;
  for (int q = 0; q < wave; ++q) run += sh[q];
  for (int64_t i = b; i < e; ++i) {
    const int32_t v = csum[i];
    csum[i] = (int32_t)run;
    run += v;
  }
}

// Scatter every entry to its block's run: lane = row, block rows start at the chunk's
// offset plus the wave's exclusive scan of the block-row lengths.
__global__ void __launch_bounds__(256)
k_split_scatter(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col, const float* __restrict__ val,
                int64_t n, int64_t bcols, const uint8_t* __restrict__ len, const int32_t* __restrict__ base,
                int64_t nch, int32_t* __restrict__ colS, float* __restrict__ valS) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; c < nch; c += waves) {
    const int64_t i = c * kSplitChunk + lane;
    int pos[kSplitBlocks];
#pragma unroll
    for (int k = 0; k < kSplitBlocks; ++k) {
      const int l = i < n ? (int)len[k * n + i] : 0;
      pos[k] = base[k * nch + c] + wave_excl_scan(l);
    }
    if (i < n) {
      const int32_t p1 = row_ptr[i + 1];
      for (int32_t p = row_ptr[i]; p < p1; ++p) {
        const int32_t j = col[p];
        const int kb = (int)((int64_t)j / bcols);
        int dst = 0;
#pragma unroll
        for (int k = 0; k < kSplitBlocks; ++k) {
          if (kb == k) {
            dst = pos[k];
            pos[k] += 1;
          }
        }
        colS[dst] = j;
        valS[dst] = val[p];
      }
    }
  }
}

// Block k's partial sum of every row: workgroup b takes block b % K and chunks
// b / K, b / K + G, ... (G = gridDim.x / K); within a wave lane l sums row c * 64 + l's
// entries of the block in order.  Terms as in the plain product (k_csr.hip).
template <int METHOD, typename T>
__global__ void __launch_bounds__(256)
k_csr_split_product(const uint8_t* __restrict__ len, const int32_t* __restrict__ base, const int32_t* __restrict__ colS,
                    const float* __restrict__ valS, int64_t n, int64_t nch, const T* __restrict__ w,
                    T* __restrict__ part, const SolveState* __restrict__ st, double alpha, double c) {
  if (state_done(st)) return;
  const int k = blockIdx.x % kSplitBlocks;
  const int64_t groups = gridDim.x / kSplitBlocks;
  const int lane = threadIdx.x & (kWave - 1);
  const int wpb = blockDim.x / kWave;
  const double ad = sizeof(T) == 4 ? (double)(float)alpha : alpha;
  const double cd = sizeof(T) == 4 ? (double)(float)c : c;
  const float af = (float)ad, cf = (float)cd;
  const uint8_t* lenk = len + (int64_t)k * n;
  const int32_t* basek = base + (int64_t)k * nch;
  T* partk = part + (int64_t)k * n;
  for (int64_t ch = (int64_t)(blockIdx.x / kSplitBlocks) * wpb + threadIdx.x / kWave; ch < nch; ch += groups * wpb) {
    const int64_t i = ch * kSplitChunk + lane;
    const int l = i < n ? (int)lenk[i] : 0;
    const int32_t p0 = basek[ch] + wave_excl_scan(l);
    T acc = T(0);
    // two entries per step: both index and value loads issue before either gather
    int e = 0;
    for (; e + 1 < l; e += 2) {
      const int32_t j0 = __builtin_nontemporal_load(colS + p0 + e);
      const int32_t j1 = __builtin_nontemporal_load(colS + p0 + e + 1);
      const float h0 = __builtin_nontemporal_load(valS + p0 + e);
      const float h1 = __builtin_nontemporal_load(valS + p0 + e + 1);
      const T w0 = w[j0], w1 = w[j1];
      if constexpr (METHOD == MAPI_METHOD_MAPI) {
        if constexpr (sizeof(T) == 4) {
          const float g0 = fmaf(af, h0, cf), g1 = fmaf(af, h1, cf);
          acc += __builtin_amdgcn_fmed3f(w0, -g0, g0) - __builtin_amdgcn_fmed3f(w0, -cf, cf);
          acc += __builtin_amdgcn_fmed3f(w1, -g1, g1) - __builtin_amdgcn_fmed3f(w1, -cf, cf);
        } else {
          const double g0 = ad * (double)h0 + cd, g1 = ad * (double)h1 + cd;
          acc += fmin(fmax(w0, -g0), g0) - fmin(fmax(w0, -cd), cd);
          acc += fmin(fmax(w1, -g1), g1) - fmin(fmax(w1, -cd), cd);
        }
      } else {
        acc = fma((T)h0, w0, acc);
        acc = fma((T)h1, w1, acc);
      }
    }
    if (e < l) {
      const int32_t j0 = __builtin_nontemporal_load(colS + p0 + e);
      const float h0 = __builtin_nontemporal_load(valS + p0 + e);
      const T w0 = w[j0];
      if constexpr (METHOD == MAPI_METHOD_MAPI) {
        if constexpr (sizeof(T) == 4) {
          const float g0 = fmaf(af, h0, cf);
          acc += __builtin_amdgcn_fmed3f(w0, -g0, g0) - __builtin_amdgcn_fmed3f(w0, -cf, cf);
        } else {
          const double g0 = ad * (double)h0 + cd;
          acc += fmin(fmax(w0, -g0), g0) - fmin(fmax(w0, -cd), cd);
        }
      } else {
        acc = fma((T)h0, w0, acc);
      }
    }
    if (i < n) partk[i] = acc;
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
         al(sizeof(float) * nnz) + al(es * kSplitBlocks * n) + al(sizeof(int32_t));
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
  return s;
}

hipError_t launch_split_count(const int32_t* row_ptr, const int32_t* col, const SplitCsr& s, hipStream_t st) {
  hipLaunchKernelGGL(k_split_count, dim3(split_grid(s.nch, 4, 16384)), dim3(256), 0, st, row_ptr, col, s.n,
                     split_block_cols(s.n), s.len, s.base, s.nch, s.flags);
  return hipGetLastError();
}

hipError_t launch_split_fill(const int32_t* row_ptr, const int32_t* col, const float* val, const SplitCsr& s,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_split_scan, dim3(1), dim3(1024), 0, st, s.base, (int64_t)kSplitBlocks * s.nch);
  hipLaunchKernelGGL(k_split_scatter, dim3(split_grid(s.nch, 4, 16384)), dim3(256), 0, st, row_ptr, col, val, s.n,
                     split_block_cols(s.n), s.len, s.base, s.nch, s.col, s.val);
  return hipGetLastError();
}

int split_combine_blocks(int64_t n) { return split_grid(n, 1024, 2048); }

template <typename T>
hipError_t launch_csr_split_product(int method, const SplitCsr& s, const T* w, T* y, double* nparts, SolveState* st,
                                    double alpha, double c, double inv_n, hipStream_t stream) {
  // 256 workgroups per column block (32 per compute unit), persistent over the chunks
  const int groups = split_grid(s.nch, 4, 256);
  const dim3 grid((unsigned)(groups * kSplitBlocks));
  T* part = static_cast<T*>(s.part);
  if (method == MAPI_METHOD_MAPI) {
    hipLaunchKernelGGL((k_csr_split_product<MAPI_METHOD_MAPI, T>), grid, dim3(256), 0, stream, s.len, s.base, s.col,
                       s.val, s.n, s.nch, w, part, st, alpha, c);
    hipLaunchKernelGGL((k_csr_split_combine<MAPI_METHOD_MAPI, T>), dim3(split_combine_blocks(s.n)), dim3(256), 0,
                       stream, part, s.n, y, nparts, st, alpha, c, inv_n);
  } else {
    hipLaunchKernelGGL((k_csr_split_product<MAPI_METHOD_RPI, T>), grid, dim3(256), 0, stream, s.len, s.base, s.col,
                       s.val, s.n, s.nch, w, part, st, alpha, c);
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
