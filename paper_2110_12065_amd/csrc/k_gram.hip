// Gram build over the rows of a data matrix X (D x N, samples as columns):
//   A_ij = scale * sum_k op(X_ik, X_jk)
// op min1/min2: the min-covariance of eq. (5), on the vector ALU (k_gram_min); op dot:
// the covariance of eq. (2), on the matrix cores (k_gram_mfma).
//
// Both builds cover the upper triangle in 128 x 128 output tiles and order their
// blocks by sample chunk first, so that the blocks resident at one time read the
// same chunk of X while it is held in the last-level cache.  Terms are summed in
// float32 within runs of 256 samples and in float64 across runs.  With several
// chunks each block writes a float64 partial tile and k_gram_reduce sums the chunks
// in order; with one chunk the block writes its tile (and the mirror) itself.  The
// chunk count depends only on D and N, so results do not depend on the device.
#include <cstdlib>
#include <cstring>

#include "common.h"

namespace mapi {

constexpr int MT = 128;          // tile edge

__device__ __forceinline__ void tile_coords(int b, int T, int* ti, int* tj) {
  int i = 0;
  while (b >= T - i) {
    b -= T - i;
    ++i;
  }
  *ti = i;
  *tj = i + b;
}

constexpr int MSP = MT + 1;      // pitch of a tile staged in LDS for its write-out

// Tile (i0, j0) of A from S (float, row pitch MSP) and, with mirror, its transpose at (j0, i0).
__device__ void gram_write_tile(const float* S, int i0, int j0, int D, float* __restrict__ A, int64_t lda, bool mirror) {
  for (int e = threadIdx.x; e < MT * MT; e += blockDim.x) {
    const int il = e / MT, jl = e % MT;
    if (i0 + il < D && j0 + jl < D) A[(int64_t)(i0 + il) * lda + j0 + jl] = S[il * MSP + jl];
  }
  if (!mirror) return;
  for (int e = threadIdx.x; e < MT * MT; e += blockDim.x) {
    const int jl = e / MT, il = e % MT;
    if (i0 + il < D && j0 + jl < D) A[(int64_t)(j0 + jl) * lda + i0 + il] = S[il * MSP + jl];
  }
}

// ---------------------------------------------------------------- min forms on the vector ALU
// Each thread holds a TM x 4 register tile of the 128 x 128 output tile: rows TM ty ..
// TM ty + TM - 1, columns 4 tx .. 4 tx + 3 (tx = tid % 32, ty = tid / 32), so that per
// sample a wave reads TM / 4 broadcast 16-byte row operands and 512 contiguous bytes of
// column operands from LDS.  TM = 4 (1024 threads, 16 waves per compute unit) is the
// build's shape: TM = 8 (512 threads) reads a quarter fewer LDS bytes per term but, at
// 163 VGPRs, leaves 8 waves per compute unit, and measured 34.1 ms against 28.9 ms for
// the min1 build at 4096 x 65536.
// X is staged through LDS in slabs of NKS samples, transposed (sample-major: the tile's
// 128 I rows then its 128 J rows, pitch NP floats), double-buffered through registers;
// the next sample's operands are read before the current sample's terms.
// min1 term: with g = |b|, med3(a, -g, g) carries min(|a|, |b|) with the sign of a, and
// sign(b) is applied by a fused multiply-add with s = +-1 (s carries the sign bit of b):
// the product is exact, so the term and the sum equal those of a sign-bit flip and an
// add, in one instruction; s is formed once per column and sample.
// min2 term: med3(a ^ signbit(b), 0, |b|) and an add, as in the product kernels.
// Every output element is summed over the samples in order, in float32 runs of 256
// samples added into float64, whatever TM: the tile shape does not change the bits.
constexpr int NKS = 32;                      // samples per slab
constexpr int NP = 2 * MT + 4;               // staged pitch (floats); 16-byte aligned
constexpr int NRUN = 256 / NKS;              // slabs per float32 run
constexpr int NLPR = NKS / 4;                // loader threads per staged row (one float4 each)
#ifndef MAPI_GRAM_TM
#define MAPI_GRAM_TM 4
#endif
#ifndef MAPI_GRAM_TN
#define MAPI_GRAM_TN 4
#endif
constexpr int kGramTM = MAPI_GRAM_TM;        // rows of a thread's register tile
constexpr int kGramTN = MAPI_GRAM_TN;        // columns of a thread's register tile (2 or 4)
constexpr int gram_threads(int tm, int tn) { return MT * MT / (tm * tn); }

// XF (min1 only): the term as the product kernels write it, a sign-bit flip of a, med3
// and an add (three instructions), instead of the FMA by +-1 (two); the same bits.
template <int OP, bool SPLIT, int TM, bool XF = false, int TN = 4>
__global__ void __launch_bounds__(gram_threads(TM, TN))
k_gram_min(const float* __restrict__ X, int D, int64_t N, int64_t ldx, int64_t chunk, int tiles, double scale,
           float* __restrict__ A, int64_t lda, double* __restrict__ part) {
  constexpr int NTH = gram_threads(TM, TN);
  constexpr int NLP = 2 * MT * NLPR / NTH;   // float4s each thread loads per slab
  constexpr int TA = TM / 4;                 // 16-byte row operands per sample
  constexpr int CT = MT / TN;                // threads along the tile's columns
  typedef float bvec __attribute__((ext_vector_type(TN)));
  __shared__ float4 lds4[2 * NKS * NP / 4];
  float* lds = reinterpret_cast<float*>(lds4);
  const int T = (D + MT - 1) / MT;
  const int tile = blockIdx.x % tiles;
  const int cidx = blockIdx.x / tiles;
  int ti, tj;
  tile_coords(tile, T, &ti, &tj);
  const int i0 = ti * MT, j0 = tj * MT;
  const int64_t kb = (int64_t)cidx * chunk;
  const int64_t ke = min(N, kb + chunk);
  const int tid = threadIdx.x, tx = tid % CT, ty = tid / CT;

  // loader: staged row sr = lrow + (NTH / NLPR) p is row sr of the I block (sr < 128)
  // or row sr - 128 of the J block; lk selects one of the slab's NLPR float4s
  const int lrow = tid / NLPR, lk = (tid % NLPR) * 4;
  float4 pre[NLP];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < NLP; ++p) {
      const int sr = lrow + (NTH / NLPR) * p;
      const int row = sr < MT ? i0 + sr : j0 + sr - MT;
      const int64_t k = k0 + lk;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (row < D) {
        const float* src = X + (int64_t)row * ldx + k;
        if (k + 3 < ke) {
          v = *reinterpret_cast<const float4*>(src);
        } else {
          if (k + 0 < ke) v.x = src[0];
          if (k + 1 < ke) v.y = src[1];
          if (k + 2 < ke) v.z = src[2];
        }
      }
      pre[p] = v;
    }
  };
  auto store = [&](int buf) {
    float* s = lds + buf * NKS * NP;
#pragma unroll
    for (int p = 0; p < NLP; ++p) {
      const int sr = lrow + (NTH / NLPR) * p;
      s[(lk + 0) * NP + sr] = pre[p].x;
      s[(lk + 1) * NP + sr] = pre[p].y;
      s[(lk + 2) * NP + sr] = pre[p].z;
      s[(lk + 3) * NP + sr] = pre[p].w;
    }
  };

  float accf[TM][TN];
  double acc[TM][TN];
#pragma unroll
  for (int p = 0; p < TM; ++p)
#pragma unroll
    for (int q = 0; q < TN; ++q) {
      accf[p][q] = 0.0f;
      acc[p][q] = 0.0;
    }

  const int64_t nslabs = (ke - kb + NKS - 1) / NKS;
  load(kb);
  store(0);
  __syncthreads();
  for (int64_t sl = 0; sl < nslabs; ++sl) {
    const int buf = (int)(sl & 1);
    if (sl + 1 < nslabs) load(kb + (sl + 1) * NKS);
    const float* s = lds + buf * NKS * NP;
    float4 a[TA];
    bvec b;
#pragma unroll
    for (int t = 0; t < TA; ++t) a[t] = *reinterpret_cast<const float4*>(s + ty * TM + 4 * t);
    b = *reinterpret_cast<const bvec*>(s + MT + tx * TN);
#pragma unroll
    for (int k = 0; k < NKS; ++k) {
      float4 an[TA];
      bvec bn;
      if (k + 1 < NKS) {
#pragma unroll
        for (int t = 0; t < TA; ++t) an[t] = *reinterpret_cast<const float4*>(s + (k + 1) * NP + ty * TM + 4 * t);
        bn = *reinterpret_cast<const bvec*>(s + (k + 1) * NP + MT + tx * TN);
      }
      float av[TM];
#pragma unroll
      for (int t = 0; t < TA; ++t) {
        av[4 * t] = a[t].x; av[4 * t + 1] = a[t].y; av[4 * t + 2] = a[t].z; av[4 * t + 3] = a[t].w;
      }
      float bv[TN];
#pragma unroll
      for (int q = 0; q < TN; ++q) bv[q] = b[q];
      if constexpr (OP == MAPI_OP_MIN1 && !XF) {
        float sg[TN];
#pragma unroll
        for (int q = 0; q < TN; ++q) sg[q] = __uint_as_float(sign_bit(bv[q]) | 0x3f800000u);
#pragma unroll
        for (int p = 0; p < TM; ++p)
#pragma unroll
          for (int q = 0; q < TN; ++q)
            accf[p][q] = fmaf(__builtin_amdgcn_fmed3f(av[p], -fabsf(bv[q]), fabsf(bv[q])), sg[q], accf[p][q]);
      } else {
        uint32_t sb[TN];
#pragma unroll
        for (int q = 0; q < TN; ++q) sb[q] = sign_bit(bv[q]);
#pragma unroll
        for (int p = 0; p < TM; ++p)
#pragma unroll
          for (int q = 0; q < TN; ++q) accf[p][q] = op_acc<OP>(accf[p][q], av[p], bv[q], sb[q]);
      }
      if (k + 1 < NKS) {
#pragma unroll
        for (int t = 0; t < TA; ++t) a[t] = an[t];
        b = bn;
      }
    }
    if ((sl + 1) % NRUN == 0 || sl + 1 == nslabs) {
#pragma unroll
      for (int p = 0; p < TM; ++p)
#pragma unroll
        for (int q = 0; q < TN; ++q) {
          acc[p][q] += (double)accf[p][q];
          accf[p][q] = 0.0f;
        }
    }
    if (sl + 1 < nslabs) {
      store(buf ^ 1);
      __syncthreads();
    }
  }

  if constexpr (SPLIT) {
    double* out = part + ((int64_t)cidx * tiles + tile) * (MT * MT);
#pragma unroll
    for (int p = 0; p < TM; ++p)
#pragma unroll
      for (int q = 0; q < TN; ++q) out[(ty * TM + p) * MT + tx * TN + q] = acc[p][q];
  } else {
    // the tile is staged in the (now free) slab buffers so that it and its mirror are
    // written along rows
    static_assert(MT * MSP <= 2 * NKS * NP, "staged tile fits the slab buffers");
    __syncthreads();
#pragma unroll
    for (int p = 0; p < TM; ++p)
#pragma unroll
      for (int q = 0; q < TN; ++q) lds[(ty * TM + p) * MSP + tx * TN + q] = (float)(scale * acc[p][q]);
    __syncthreads();
    gram_write_tile(lds, i0, j0, D, A, lda, ti != tj);
  }
}

// ---------------------------------------------------------------- covariance on the matrix cores
// The dot form (eq. 2 covariance, the RPI build) is a dense contraction and runs on
// v_mfma_f32_32x32x2f32; the min forms have no product and stay on the vector ALU.
//
// Upper-triangle 128 x 128 output tiles, 512 threads: wave (wr, wc) of 8 owns rows
// 32 wr .. 32 wr + 31 and columns 64 wc .. 64 wc + 63 of the tile as two 32 x 32
// accumulators.  For this instruction lane l supplies A[l % 32][l / 32] and
// B[l / 32][l % 32] and holds C[8 (v / 4) + 4 (l / 32) + v % 4][l % 32] in accumulator
// register v.  X is staged through LDS in slabs of MKS samples of the tile's 128 + 128
// rows (each row padded by 4 floats: a pitch of an odd number of 16-byte units puts the
// 16-byte reads of 16 consecutive rows on distinct banks), double-buffered through
// registers.  Half h of a wave takes samples (MKS / 2) h .. (MKS / 2) (h + 1) - 1 of a
// slab, so one 16-byte LDS read feeds four MFMA steps, and the two halves' terms in a
// step are two samples of the same pair of rows.  The float32 runs are the matrix
// cores' own adds.
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int MKS = 64;         // samples per LDS slab
constexpr int MROW = MKS + 4;   // staged row pitch (floats): an odd number of 16-byte units
constexpr int MRUN = 256 / MKS; // slabs per float32 run (256 samples)
constexpr int MLPR = MKS / 4;   // loader threads per staged row (one float4 each)
constexpr int MLP = 2 * MT * MLPR / 512;   // float4s each of the 512 threads loads per slab

template <bool SPLIT>
__global__ void __launch_bounds__(512)
k_gram_mfma(const float* __restrict__ X, int D, int64_t N, int64_t ldx, int64_t chunk, int tiles, double scale,
            float* __restrict__ A, int64_t lda, double* __restrict__ part) {
  __shared__ float4 lds4[2 * 2 * MT * MROW / 4];
  float* lds = reinterpret_cast<float*>(lds4);
  const int T = (D + MT - 1) / MT;
  const int tile = blockIdx.x % tiles;
  const int cidx = blockIdx.x / tiles;
  int ti, tj;
  tile_coords(tile, T, &ti, &tj);
  const int i0 = ti * MT, j0 = tj * MT;
  const int64_t kb = (int64_t)cidx * chunk;
  const int64_t ke = min(N, kb + chunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int h = lane >> 5, r = lane & 31;

  // loader: staged row sr = lrow + (512 / MLPR) p is row sr of the I block (sr < 128)
  // or row sr - 128 of the J block; lk selects one of the slab's MLPR float4s
  const int lrow = tid / MLPR, lk = (tid % MLPR) * 4;
  float4 pre[MLP];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < MLP; ++p) {
      const int sr = lrow + (512 / MLPR) * p;
      const int row = sr < MT ? i0 + sr : j0 + sr - MT;
      const int64_t k = k0 + lk;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (row < D) {
        const float* src = X + (int64_t)row * ldx + k;
        if (k + 3 < ke) {
          v = *reinterpret_cast<const float4*>(src);
        } else {
          if (k + 0 < ke) v.x = src[0];
          if (k + 1 < ke) v.y = src[1];
          if (k + 2 < ke) v.z = src[2];
        }
      }
      pre[p] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int p = 0; p < MLP; ++p)
      *reinterpret_cast<float4*>(lds + (buf * 2 * MT + lrow + (512 / MLPR) * p) * MROW + lk) = pre[p];
  };

  f32x16 acc0 = {}, acc1 = {};
  double d0[16], d1[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) d0[v] = d1[v] = 0.0;

  const int64_t nslabs = (ke - kb + MKS - 1) / MKS;
  load(kb);
  store(0);
  __syncthreads();
  for (int64_t sl = 0; sl < nslabs; ++sl) {
    const int buf = (int)(sl & 1);
    if (sl + 1 < nslabs) load(kb + (sl + 1) * MKS);
    const float* pa = lds + (buf * 2 * MT + wr * 32 + r) * MROW + (MKS / 2) * h;
    const float* pb = lds + (buf * 2 * MT + MT + wc * 64 + r) * MROW + (MKS / 2) * h;
#pragma unroll
    for (int q = 0; q < MKS / 8; ++q) {
      const float4 a = *reinterpret_cast<const float4*>(pa + 4 * q);
      const float4 b0 = *reinterpret_cast<const float4*>(pb + 4 * q);
      const float4 b1 = *reinterpret_cast<const float4*>(pb + 32 * MROW + 4 * q);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b0.x, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b1.x, acc1, 0, 0, 0);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b0.y, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b1.y, acc1, 0, 0, 0);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b0.z, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b1.z, acc1, 0, 0, 0);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b0.w, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b1.w, acc1, 0, 0, 0);
    }
    if ((sl + 1) % MRUN == 0 || sl + 1 == nslabs) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        d0[v] += (double)acc0[v];
        d1[v] += (double)acc1[v];
      }
      acc0 = f32x16{};
      acc1 = f32x16{};
    }
    if (sl + 1 < nslabs) {
      store(buf ^ 1);
      __syncthreads();
    }
  }

  // accumulator register v of tile t: row 32 wr + 8 (v / 4) + 4 h + v % 4, column 64 wc + 32 t + r
  if constexpr (SPLIT) {
    double* out = part + ((int64_t)cidx * tiles + tile) * (MT * MT);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int il = wr * 32 + (v >> 2) * 8 + h * 4 + (v & 3);
      out[il * MT + wc * 64 + r] = d0[v];
      out[il * MT + wc * 64 + 32 + r] = d1[v];
    }
  } else {
    __syncthreads();      // the staging buffers are reused for the output tile
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int il = wr * 32 + (v >> 2) * 8 + h * 4 + (v & 3);
      lds[il * MSP + wc * 64 + r] = (float)(scale * d0[v]);
      lds[il * MSP + wc * 64 + 32 + r] = (float)(scale * d1[v]);
    }
    __syncthreads();
    gram_write_tile(lds, i0, j0, D, A, lda, ti != tj);
  }
}

// Sum of the KC float64 partial tiles in chunk order, scaled and rounded once.
__global__ void __launch_bounds__(256)
k_gram_reduce(const double* __restrict__ part, int kc, int tiles, int D, double scale, float* __restrict__ A,
              int64_t lda) {
  __shared__ float S[MT * MSP];
  const int T = (D + MT - 1) / MT;
  int ti, tj;
  tile_coords(blockIdx.x, T, &ti, &tj);
  for (int e = threadIdx.x; e < MT * MT; e += blockDim.x) {
    double sum = 0.0;
    for (int c = 0; c < kc; ++c) sum += part[((int64_t)c * tiles + blockIdx.x) * (MT * MT) + e];
    S[(e / MT) * MSP + e % MT] = (float)(scale * sum);
  }
  __syncthreads();
  gram_write_tile(S, ti * MT, tj * MT, D, A, lda, ti != tj);
}

// Sample chunks of a Gram build: the KC in 1..kc_max (at most one per 256-sample run)
// that minimises rounds of `resident` blocks per chunk of work.  resident is the
// block count one launch keeps on the chip (a constant per kernel, not read from the
// device, so that the chunking and with it the result depend only on D and N).
struct GramSplit {
  int64_t tiles, chunk;
  int kc;
};
static GramSplit gram_split(int64_t D, int64_t N, int64_t resident, int kc_max) {
  const int64_t T = (D + MT - 1) / MT, tiles = T * (T + 1) / 2;
  const int64_t runs = (N + 255) / 256;
  int best = 1;
  double best_cost = 1e300;
  for (int kc = 1; kc <= kc_max && kc <= runs; ++kc) {
    const double cost = (double)((tiles * kc + resident - 1) / resident) / kc;
    if (cost < best_cost - 1e-12) {
      best_cost = cost;
      best = kc;
    }
  }
  const int64_t chunk = (runs + best - 1) / best * 256;
  return GramSplit{tiles, chunk, (int)((N + chunk - 1) / chunk)};
}
// one block per CU for both builds
static GramSplit gram_split_op(int64_t D, int64_t N, int op) {
  return op == MAPI_OP_DOT ? gram_split(D, N, 256, 8) : gram_split(D, N, 256, 16);
}

size_t gram_workspace_bytes(int64_t D, int64_t N, int op) {
  const GramSplit g = gram_split_op(D, N, op);
  return g.kc > 1 ? (size_t)g.kc * (size_t)g.tiles * MT * MT * sizeof(double) : 0;
}

template <int OP, bool XF = false>
static void launch_gram_min(const GramSplit& g, const float* X, int64_t D, int64_t N, int64_t ldx, double scale,
                            float* A, int64_t lda, double* ws, hipStream_t s) {
  constexpr int NTH = gram_threads(kGramTM, kGramTN);
  if (g.kc > 1)
    hipLaunchKernelGGL((k_gram_min<OP, true, kGramTM, XF, kGramTN>), dim3((unsigned)(g.tiles * g.kc)), dim3(NTH), 0,
                       s, X, (int)D, N, ldx, g.chunk, (int)g.tiles, scale, A, lda, ws);
  else
    hipLaunchKernelGGL((k_gram_min<OP, false, kGramTM, XF, kGramTN>), dim3((unsigned)g.tiles), dim3(NTH), 0, s, X,
                       (int)D, N, ldx, g.chunk, (int)g.tiles, scale, A, lda, nullptr);
}

// MAPI_MIN1_FORM=xor selects the three-instruction min1 term (for comparison; the
// result has the same bits), read at each build.
bool min1_xor_form() {
  const char* e = std::getenv("MAPI_MIN1_FORM");
  return e != nullptr && std::strcmp(e, "xor") == 0;
}

hipError_t launch_gram(const float* X, int64_t D, int64_t N, int64_t ldx, double scale, int op, float* A, int64_t lda,
                       double* ws, hipStream_t s) {
  if (op != MAPI_OP_DOT && op != MAPI_OP_MIN1 && op != MAPI_OP_MIN2) return hipErrorInvalidValue;
  const GramSplit g = gram_split_op(D, N, op);
  if (g.kc > 1 && !ws) return hipErrorInvalidValue;
  if (op == MAPI_OP_DOT) {
    if (g.kc > 1)
      hipLaunchKernelGGL(k_gram_mfma<true>, dim3((unsigned)(g.tiles * g.kc)), dim3(512), 0, s, X, (int)D, N, ldx,
                         g.chunk, (int)g.tiles, scale, A, lda, ws);
    else
      hipLaunchKernelGGL(k_gram_mfma<false>, dim3((unsigned)g.tiles), dim3(512), 0, s, X, (int)D, N, ldx, g.chunk,
                         (int)g.tiles, scale, A, lda, nullptr);
  } else if (op == MAPI_OP_MIN1) {
    if (min1_xor_form()) launch_gram_min<MAPI_OP_MIN1, true>(g, X, D, N, ldx, scale, A, lda, ws, s);
    else launch_gram_min<MAPI_OP_MIN1>(g, X, D, N, ldx, scale, A, lda, ws, s);
  } else {
    launch_gram_min<MAPI_OP_MIN2>(g, X, D, N, ldx, scale, A, lda, ws, s);
  }
  if (g.kc > 1)
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)g.tiles), dim3(256), 0, s, ws, g.kc, (int)g.tiles, (int)D, scale,
                       A, lda);
  return hipGetLastError();
}

// ---------------------------------------------------------------- deflation
// Vector i is extracted from (I - P P^T) A = A - P Q with Q = P^T A (P
// orthonormal, float64).  Q gains one row per extracted vector.

// q_j = sum_i p_i A_ij for one new column p of P: column sums of a row-weighted
// A, reduced over row chunks into `qpart` and then in a fixed order.
constexpr int QCH = 64;   // row chunks

__global__ void __launch_bounds__(256)
k_deflate_qpart(const float* __restrict__ A, int64_t D, int64_t lda, const double* __restrict__ p,
                double* __restrict__ qpart) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int chunk = blockIdx.y;
  const int64_t rows = (D + QCH - 1) / QCH;
  const int64_t r0 = chunk * rows, r1 = min(D, r0 + rows);
  if (j >= D) return;
  double s = 0.0;
  for (int64_t i = r0; i < r1; ++i) s += p[i] * (double)A[i * lda + j];
  qpart[(int64_t)chunk * D + j] = s;
}

__global__ void k_deflate_qsum(const double* __restrict__ qpart, int64_t D, double* __restrict__ q) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= D) return;
  double s = 0.0;
  for (int c = 0; c < QCH; ++c) s += qpart[(int64_t)c * D + j];
  q[j] = s;
}

// out_ij = fl32(A_ij - sum_l P_il Q_lj), float64 arithmetic.  P: D x k column-major; Q: k x D row-major.
__global__ void __launch_bounds__(256)
k_deflate_apply(const float* __restrict__ A, int64_t D, int64_t lda, const double* __restrict__ P,
                const double* __restrict__ Q, int k, float* __restrict__ out, int64_t ldo) {
  const int64_t i = blockIdx.y;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < D; j += (int64_t)gridDim.x * blockDim.x) {
    double v = (double)A[i * lda + j];
    for (int l = 0; l < k; ++l) v -= P[(int64_t)l * D + i] * Q[(int64_t)l * D + j];
    out[i * ldo + j] = (float)v;
  }
}

// Append w to P: p = w / ||w||_2, then modified Gram-Schmidt against the k
// existing columns, then normalise again; writes P[:, k] (float64) and p_out (float32).
__global__ void __launch_bounds__(1024)
k_mgs_append(double* __restrict__ P, int64_t D, int k, const float* __restrict__ w, float* __restrict__ p_out) {
  __shared__ double sh[16];
  double* pk = P + (int64_t)k * D;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < D; i += blockDim.x) {
    const double v = (double)w[i];
    pk[i] = v;
    s += v * v;
  }
  s = block_sum_f64(s, sh);
  double inv = 1.0 / sqrt(s);
  for (int64_t i = threadIdx.x; i < D; i += blockDim.x) pk[i] *= inv;
  __syncthreads();
  for (int l = 0; l < k; ++l) {
    const double* pl = P + (int64_t)l * D;
    double d = 0.0;
    for (int64_t i = threadIdx.x; i < D; i += blockDim.x) d += pl[i] * pk[i];
    d = block_sum_f64(d, sh);
    for (int64_t i = threadIdx.x; i < D; i += blockDim.x) pk[i] -= d * pl[i];
    __syncthreads();
  }
  s = 0.0;
  for (int64_t i = threadIdx.x; i < D; i += blockDim.x) s += pk[i] * pk[i];
  s = block_sum_f64(s, sh);
  inv = 1.0 / sqrt(s);
  for (int64_t i = threadIdx.x; i < D; i += blockDim.x) {
    pk[i] *= inv;
    p_out[i] = (float)pk[i];
  }
}

hipError_t launch_deflate_q(const float* A, int64_t D, int64_t lda, const double* p, double* q, double* qpart,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_deflate_qpart, dim3((unsigned)((D + 255) / 256), QCH), dim3(256), 0, s, A, D, lda, p, qpart);
  hipLaunchKernelGGL(k_deflate_qsum, dim3((unsigned)((D + 255) / 256)), dim3(256), 0, s, qpart, D, q);
  return hipGetLastError();
}

hipError_t launch_deflate_apply(const float* A, int64_t D, int64_t lda, const double* P, const double* Q, int k,
                                float* out, int64_t ldo, hipStream_t s) {
  const unsigned gx = (unsigned)((D + 255) / 256 < 16 ? (D + 255) / 256 : 16);
  hipLaunchKernelGGL(k_deflate_apply, dim3(gx, (unsigned)D), dim3(256), 0, s, A, D, lda, P, Q, k, out, ldo);
  return hipGetLastError();
}

hipError_t launch_mgs_append(double* P, int64_t D, int k, const float* w, float* p_out, hipStream_t s) {
  hipLaunchKernelGGL(k_mgs_append, dim3(1), dim3(1024), 0, s, P, D, k, w, p_out);
  return hipGetLastError();
}

int deflate_qpart_count() { return QCH; }

}  // namespace mapi
