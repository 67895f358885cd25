// Shared device helpers and launcher declarations of libmapi (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mapi.h"
#include "ops.h"

namespace mapi {

constexpr int kWave = 64;

// Device-resident state of one power-iteration solve.  Kernels read `done` on
// entry and return at once when it is set, so a host loop may enqueue more
// iterations than are needed and poll rarely.
struct SolveState {
  double nu;          // normaliser of the latest product (l1 or l2)
  double r;           // residual ||w_t - w_{t-1}||_1 of the latest iteration
  double best_r;      // smallest residual so far (stall rule)
  double ex[2];       // PageRank scalars of the current iterate
  double tol;
  int32_t iter;       // completed iterations
  int32_t done;
  int32_t converged;
  int32_t status;     // mapi_status of the solve
  int32_t stall;
  int32_t max_iters;
  int32_t stall_iters;
  uint32_t check;     // device-checked builds: the first failed check (file id << 16 | line)
  uint32_t cnt_b;     // arrival counter of the normalisation kernel's reduction
  int32_t pad;
};

enum NormKind { NORM_NONE = 0, NORM_L1 = 1, NORM_L2 = 2 };

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Cross-lane moves within rows of 16 lanes (DPP, no LDS round trip): quad_perm xor 1
// and xor 2, row_half_mirror (lane i of each 8 from lane 7 - i) and row_mirror (lane i
// of each 16 from lane 15 - i).
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// v(lane) + v(lane ^ B) for B = 16 or 32 by a lane swap of v with itself (both words).
template <int B>
__device__ __forceinline__ double swap_pair_sum(double v) {
  const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
  const auto a = B == 32 ? __builtin_amdgcn_permlane32_swap(lo, lo, false, false)
                         : __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = B == 32 ? __builtin_amdgcn_permlane32_swap(hi, hi, false, false)
                         : __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}

// Sum over the wave, the same bits in every lane (each step adds the same two values on
// both sides of a pair): quads, 8s and 16s by DPP, then lane bits 4 and 5 by lane swaps.
__device__ __forceinline__ double wave_total_f64(double v) {
  v += dpp_f64<kDppXor1>(v);
  v += dpp_f64<kDppXor2>(v);
  v += dpp_f64<kDppHalfMirror>(v);
  v += dpp_f64<kDppMirror>(v);
  v = swap_pair_sum<16>(v);
  v = swap_pair_sum<32>(v);
  return v;
}

// Fixed-order block sum of one double per thread (blockDim.x <= 1024).  Result
// valid in every thread.  `sh` holds at least blockDim.x / 64 doubles.
__device__ __forceinline__ double block_sum_f64(double v, double* sh) {
  v = wave_sum_f64(v);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += sh[i];
  return s;
}

__device__ __forceinline__ void store_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_agent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Fixed-order sum of part[0..count) by one wave (lane l adds l, l + 64, ... in that
// order; then a butterfly): every wave that calls it gets the same bits, whatever the
// block size, so the normaliser is identical in every kernel that forms it.  The
// partials were written by an earlier launch (visible from kernel start): plain loads,
// four per lane in flight, so that the sum costs one memory round trip per 256 partials.
__device__ __forceinline__ double wave_sum_parts(const double* part, int count) {
  const int lane = threadIdx.x & (kWave - 1);
  double s = 0.0;
  int i = lane;
  for (; i + 3 * kWave < count; i += 4 * kWave) {
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = part[i + k * kWave];
#pragma unroll
    for (int k = 0; k < 4; ++k) s += v[k];
  }
  for (; i < count; i += kWave) s += part[i];
  return wave_sum_f64(s);
}

// Publish this block's partial(s) and report whether it arrived last.  The
// last block then sees every other block's partials.  Call from all threads.
__device__ __forceinline__ bool arrive_last(uint32_t* counter, int* sh_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t prev = atomicAdd(counter, 1u);
    *sh_flag = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  const bool last = *sh_flag != 0;
  if (last) __threadfence();
  return last;
}

// Fixed-order sum of part[0..count) (stride `stride`, offset `off`) by one block.
__device__ __forceinline__ double block_sum_parts(const double* part, int count, int stride, int off,
                                                  double* sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) s += load_agent(&part[(size_t)i * stride + off]);
  return block_sum_f64(s, sh);
}

// Device checks.  In a build with MAPI_DEVICE_CHECKS (libmapi_checked.so) MAPI_DCHECK(st,
// cond, file_id) evaluates cond and, when it fails, records file_id << 16 | line in st->check
// (the first failure is kept) and yields false, so that the caller skips or clamps the
// access it guards and the kernel still ends normally; the host turns a recorded failure
// into MAPI_ERR_DEVICE_CHECK.  In the ordinary build it is the constant true.
// File ids: 1 dense product, 2 CSR product, 3 column-split product, 4 batched kernel.
__device__ __forceinline__ void dcheck_fail(const SolveState* st, uint32_t file_id, uint32_t line) {
  if (st != nullptr) atomicCAS(const_cast<uint32_t*>(&st->check), 0u, (file_id << 16) | (line & 0xFFFFu));
}
#ifdef MAPI_DEVICE_CHECKS
#define MAPI_DCHECK(st, cond, file_id) ((cond) ? true : (::mapi::dcheck_fail((st), (file_id), __LINE__), false))
#else
#define MAPI_DCHECK(st, cond, file_id) true
#endif

__device__ __forceinline__ bool state_done(const SolveState* st) {
  return __hip_atomic_load(const_cast<int32_t*>(&st->done), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Advance the stop rule after an iteration's residual r is known (one thread).
__device__ __forceinline__ void state_advance(SolveState* st, double r) {
  st->iter += 1;
  st->r = r;
  if (r < st->tol) {
    st->converged = 1;
    st->done = 1;
  } else if (st->iter >= st->max_iters) {
    st->done = 1;
  } else if (st->stall_iters > 0) {
    if (r < st->best_r) {
      st->best_r = r;
      st->stall = 0;
    } else if (++st->stall >= st->stall_iters) {
      st->done = 1;
    }
  }
}

// wave_sum_parts in two steps, so that other loads can be issued between the partials'
// loads and their sum: parts_load loads lane l's first kPartsPre partials (l, l + 64,
// ...), parts_sum adds them and any further ones in the same order as wave_sum_parts
// (the same bits).
constexpr int kPartsPre = 8;
__device__ __forceinline__ void parts_load(const double* part, int count, double* v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int k = 0; k < kPartsPre; ++k) {
    const int i = lane + k * kWave;
    v[k] = i < count ? part[i] : 0.0;
  }
}
__device__ __forceinline__ double parts_sum(const double* part, int count, const double* v) {
  const int lane = threadIdx.x & (kWave - 1);
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kPartsPre; ++k)
    if (lane + k * kWave < count) s += v[k];
  for (int i = lane + kPartsPre * kWave; i < count; i += kWave) s += part[i];
  return wave_sum_f64(s);
}

// The stop rule's inputs as a kernel found them, read by the one thread that will
// advance the rule together with the kernel's other first loads, so that advancing
// it later waits for no memory round trip.
struct StopSnap {
  double best_r, tol;
  int32_t iter, stall, max_iters, stall_iters;
};
__device__ __forceinline__ StopSnap stop_snap(const SolveState* st) {
  return StopSnap{st->best_r, st->tol, st->iter, st->stall, st->max_iters, st->stall_iters};
}
// state_advance on a snapshot of a state that no other thread changes meanwhile; returns
// whether the solve is done now.
__device__ __forceinline__ bool state_advance_from(SolveState* st, const StopSnap& s, double r) {
  const int32_t iter = s.iter + 1;
  st->iter = iter;
  st->r = r;
  if (r < s.tol) {
    st->converged = 1;
    st->done = 1;
    return true;
  }
  if (iter >= s.max_iters) {
    st->done = 1;
    return true;
  }
  if (s.stall_iters > 0) {
    if (r < s.best_r) {
      st->best_r = r;
      st->stall = 0;
    } else {
      st->stall = s.stall + 1;
      if (s.stall + 1 >= s.stall_iters) {
        st->done = 1;
        return true;
      }
    }
  }
  return false;
}

// ---------------------------------------------------------------- launchers
struct DenseArgs {
  const void* A;
  int64_t ld;
  int64_t n_rows, n_cols;
  int32_t dtype;
  const float* row_scale;
  hipEvent_t ev_start = nullptr;   // when set, attached to the launch's dispatch (kernel time)
  hipEvent_t ev_stop = nullptr;
  int reverse = 0;                 // sweep the rows in mirrored order (see k_mavp_dense)
};

struct DenseTuning {
  int rows_per_wave;   // 1, 2, 4 or 8 rows share each staged w value
  int waves;           // waves per block (4 or 8)
  int blocks;          // grid size (persistent loop over row groups); 0 = from blocks_per_cu
  int w_in_lds;        // 0: w from global memory; 1: w staged in LDS; 2 (FP8 only): |w| and sign words in LDS
  int blocks_per_cu;   // grid = CUs * blocks_per_cu (0 = default)
  int unroll;          // 16-byte loads in flight per row per lane (2 or 4)
  int nontemporal;     // non-temporal matrix loads
};

// LDS bytes of the dense product kernel for a w_in_lds mode: w (mode 1) or |w|
// plus one sign word per 4 columns (mode 2, FP8 storage).
// Floats of w staged in LDS: whole 16-byte matrix vectors (VE = 16 / element
// size columns each), padded to groups of 64 vectors for the chunk-interleaved order.
__host__ __device__ inline int64_t dense_lds_w_floats(int dtype, int64_t n_cols) {
  const int64_t ve = dtype == MAPI_FP8_E4M3 ? 16 : (dtype == MAPI_BF16 ? 8 : 4);
  return (n_cols / ve + 63) / 64 * 64 * ve;
}
// The columns past the last whole vector (fewer than 16) follow the staged
// vectors in kDenseTailFloats floats when the product forms w itself (FusedPrev).
constexpr int kDenseTailFloats = 16;
inline size_t dense_lds_bytes(int dtype, int64_t n_cols, int mode) {
  const size_t wbytes = (size_t)(dense_lds_w_floats(dtype, n_cols) + kDenseTailFloats) * 4;
  if (mode == 0) return 0;
  return (mode == 2 && dtype == MAPI_FP8_E4M3) ? wbytes + (size_t)((n_cols >> 2) + 4) * 4 : wbytes;
}

// Normalisation and convergence check of the previous iteration folded into a
// dense product.  Launch t (t >= 1) forms nu_t from the previous product's
// partials, stages w_t = y_t * (1 / nu_t) in LDS instead of reading w, writes its
// share of w_t to w_new and adds |w_t - w_{t-1}| over that share (w_old) into a
// float64 residual partial (rpart_out, one per block).  The residual of iteration
// t is therefore known only to the next launch, which sums rpart_prev in a fixed
// order and advances the stop rule for iteration t - 1 before anything else: the
// stop decision lags one launch, and a solve that converges at iteration t has
// computed one product past it.  A zero or non-finite nu marks the solve
// degenerate after `iter` - 1 completed iterations.
struct FusedPrev {
  const float* y_prev;
  const double* part_prev;
  int nparts;
  float* w_new;
  int iter;
  const float* w_old;          // w_{t-1}
  const double* rpart_prev;    // residual partials of iteration t - 1 (NULL for t = 1)
  double* rpart_out;           // residual partials of iteration t
};
// Admissible w_in_lds modes for a storage type.
inline bool lds_mode_ok(int dtype, int mode) { return mode == 0 || mode == 1 || (mode == 2 && dtype == MAPI_FP8_E4M3); }

hipError_t launch_state_init(SolveState* st, int max_iters, double tol, int stall_iters, hipStream_t s);
hipError_t launch_mavp_dense(const DenseArgs& a, int op, const float* w, float* y, double* part,
                             SolveState* st, int norm, const DenseTuning& t, int cu_count, hipStream_t s,
                             const FusedPrev* fp = nullptr);
int dense_part_count(const DenseArgs& a, const DenseTuning& t, int cu_count);
DenseTuning dense_default_tuning(const DenseArgs& a, int cu_count, int max_lds_bytes);
// rprev (dense only): residual partials of the previous iteration, written by a
// product that formed that iterate (FusedPrev); they are summed and the stop rule
// advanced for that iteration before this one is formed.
hipError_t launch_finalize(int mode, const float* y, const float* w_old, float* w_new, int64_t n,
                           SolveState* st, const double* pprod, int nprod, int norm, double* part,
                           const uint8_t* dangling, double c, double inv_n, hipStream_t s,
                           const double* rprev = nullptr, int nrprev = 0);
// The same for a float64 iterate (PageRank modes 1 and 2).
hipError_t launch_finalize_f64(int mode, const double* y, const double* w_old, double* w_new, int64_t n,
                               SolveState* st, const double* pprod, int nprod, double* part, const uint8_t* dangling,
                               double c, double inv_n, hipStream_t s);
int finalize_blocks(int64_t n);
// Whole solve of a small dense float32 system in one block (n <= 256): the state must
// be initialised; writes the final iterate (optional l2 step) to out and the state.
bool small_solve_fits(int64_t n, int op);
constexpr int kSmallMaxIters = 1 << 16;   // longer solves launch per iteration
hipError_t launch_solve_small(int op, const float* A, int64_t ld, int64_t n, const float* w0, float* out,
                              SolveState* st, int norm, int final_l2, hipStream_t s);
// Vectors of more than 65536 elements use many blocks; `part` (device, at least
// min(256, ceil(n / 4096)) doubles, free for this use) then holds their partial sums.
hipError_t launch_finish(const float* w0buf, const float* w1buf, float* out, int64_t n, SolveState* st, int final_l2,
                         hipStream_t s, double* part = nullptr);
hipError_t launch_finish_f64(const double* w0buf, const double* w1buf, double* out, int64_t n, SolveState* st,
                             int final_l2, hipStream_t s, double* part = nullptr);

hipError_t launch_quant_bf16(const float* A, int64_t n_rows, int64_t n_cols, int64_t lda, uint16_t* out,
                             int64_t ldo, hipStream_t s);
hipError_t launch_quant_fp8(const float* A, int64_t n_rows, int64_t n_cols, int64_t lda, uint8_t* out,
                            int64_t ldo, float* scale, hipStream_t s);

// Gram build (eq. 5 min forms, eq. 2 dot); ws: gram_workspace_bytes(D, N, op) bytes
// of device memory (float64 partial tiles of the covariance build), or NULL when that is 0.
size_t gram_workspace_bytes(int64_t D, int64_t N, int op);
hipError_t launch_gram(const float* X, int64_t D, int64_t N, int64_t ldx, double scale, int op, float* A,
                       int64_t lda, double* ws, hipStream_t s);

hipError_t launch_csr_prep(const int32_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz, uint8_t* dangling,
                           int32_t* err, hipStream_t s);
// PageRank kernels for a float32 or float64 iterate T (instantiated for both).
template <typename T>
hipError_t launch_pr_scalars(int method, const T* w, int64_t n, const uint8_t* dangling, double c, double inv_n,
                             SolveState* st, double* part, hipStream_t s);
template <typename T>
hipError_t launch_csr_product(int method, const int32_t* row_ptr, const int32_t* col, const float* val, int64_t n,
                              const T* w, T* y, double* part, SolveState* st, double alpha, double c, double inv_n,
                              hipStream_t s);
int csr_part_count(int64_t n);

// Column-split copy of a CSR link matrix (k_csr_split.hip): the entries of each of 8
// source blocks contiguous, per-row lengths per block, per-chunk offsets, and the
// products' per-block partial row sums.
struct SplitCsr {
  int64_t n = 0, nnz = 0, nch = 0;
  uint8_t* len = nullptr;
  int32_t* base = nullptr;
  int32_t* col = nullptr;
  float* val = nullptr;
  void* part = nullptr;
  int32_t* flags = nullptr;
  int32_t* deg = nullptr;      // estimated links per source (hub ranking)
  int32_t* slot = nullptr;     // LDS slot of a hub source, -1 otherwise
  int32_t* hubs = nullptr;     // hub sources per block, by slot
  int32_t* nhub = nullptr;     // hubs per block
  int32_t* thr = nullptr;      // hub degree threshold per block
  int32_t* hist = nullptr;     // degree histogram per block
  void* hval = nullptr;        // iterate values of the hubs per block, by slot (per product)
  int32_t* tsum = nullptr;     // tile sums of the offset scan
};
// Device bytes of the split copy for an iterate of es bytes per element, and its placement.
size_t split_csr_bytes(int64_t n, int64_t nnz, size_t es);
SplitCsr split_csr_place(void* ws, int64_t n, int64_t nnz, size_t es);
// Count block-row lengths (flags must be zero; bit 0 set when a block row is too long for
// the split layout), then, only if it is not, fill the offsets and the split entries.
hipError_t launch_split_count(const int32_t* row_ptr, const int32_t* col, const float* val, const SplitCsr& s,
                              hipStream_t st);
hipError_t launch_split_fill(const int32_t* row_ptr, const int32_t* col, const float* val, const SplitCsr& s,
                             hipStream_t st);
// Normaliser partials written by the split product (its combine kernel's grid).
int split_combine_blocks(int64_t n);
// One split product: the per-block partial sums, then y and the normaliser partials.
template <typename T>
hipError_t launch_csr_split_product(int method, const SplitCsr& s, const T* w, T* y, double* nparts, SolveState* st,
                                    double alpha, double c, double inv_n, hipStream_t stream);

hipError_t launch_deflate_q(const float* A, int64_t D, int64_t lda, const double* p, double* q, double* qpart,
                            hipStream_t s);
int deflate_qpart_count();
hipError_t launch_deflate_apply(const float* A, int64_t D, int64_t lda, const double* P, const double* Q, int k,
                                float* out, int64_t ldo, hipStream_t s);
hipError_t launch_mgs_append(double* P, int64_t D, int k, const float* w, float* p_out, hipStream_t s);
int pr_scalar_blocks(int64_t n);
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);
hipError_t launch_copy16(const void* src, void* dst, int64_t n16, int cu_count, hipStream_t s);
// MAPI_MIN1_FORM=xor in the environment: the min-Gram build and the one-block solve write
// the min1 term as sign flip, med3 and add instead of med3 and an FMA by +-1 (k_gram.hip).
bool min1_xor_form();
// One always-failing device check on st (a no-op outside device-checked builds).
hipError_t launch_dcheck_selftest(SolveState* st, hipStream_t s);
// Start vector of the generated problem with this seed (k_batched.hip).
hipError_t launch_gen_start(int n, uint64_t seed, float* w, hipStream_t s);
hipError_t launch_read16(const void* src, int64_t n16, uint32_t* sink, int blocks, int unroll, hipStream_t s);

int image_max_n();
hipError_t launch_img_center(const float* V, int64_t P, int N, int64_t ldv, float* Vc, int64_t ldc, float* m,
                             hipStream_t s);
// Doubles of the deflation's segment sums per (segment, column): sums holds G * P times this.
int image_defl_sums_per_column();
hipError_t launch_img_minouter_deflate(int op, const float* C, int64_t P, int64_t ldc, const float* w, int32_t* perm,
                                       double* sums, int G, float* Cd, hipStream_t s);
hipError_t launch_img_reconstruct(int op, const float* W, const float* Vc, int64_t P, int N, int64_t ldc,
                                  const float* m, float* R, int64_t ldr, hipStream_t s);

// Column products z = X^T (+) w (op MIN1 or MIN2) of the factored operator: RC =
// col_product_chunks(D) row chunks written to zpart (RC x N floats), then summed in
// chunk order into z (N floats).  Skipped once the solve state is done.
int col_product_chunks(int64_t D);
hipError_t launch_col_product(int op, const float* X, int64_t D, int64_t N, int64_t ldx, const float* w,
                              float* zpart, float* z, const SolveState* st, hipStream_t s);

// Per-run outcome of the mini-batch kernel.
struct MbRun {
  int32_t iters, status;
  double nu;       // last normaliser
};
int minibatch_max_d();
// Steps of t whose batch matrices are built ahead in one launch (at most 256 MiB of them).
int minibatch_range(int D, int T, int runs);
// Device workspace of launch_minibatch: the stored batch matrices of `range` steps of t
// and a state record per run.
size_t minibatch_workspace_bytes(int D, int range, int runs);
hipError_t launch_minibatch(const float* X, int64_t N, int D, int64_t ldx, const int32_t* idx, int s, int T, float beta,
                            int op, int runs, const float* w0, float* w_out, int final_l2, MbRun* run_info,
                            int32_t* bad_index, int range, void* ws, hipStream_t st);

}  // namespace mapi
