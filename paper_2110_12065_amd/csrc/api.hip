// C-ABI of libmapi: argument checks, device workspace, iteration drivers and
// kernel timing.  Declarations and contracts are in include/mapi.h.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>


#include "ctx.h"

using namespace mapi;

namespace mapi {

thread_local std::string g_err;

mapi_status fail(mapi_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

}  // namespace mapi

namespace {

mapi_status check_dense(const mapi_dense* A, bool square) {
  if (!A || !A->data) return fail(MAPI_ERR_ARG, "matrix descriptor or data pointer is NULL");
  if (A->n_rows <= 0 || A->n_cols <= 0) return fail(MAPI_ERR_ARG, "matrix is empty (%lld x %lld)",
                                                    (long long)A->n_rows, (long long)A->n_cols);
  if (A->n_rows > INT32_MAX || A->n_cols > INT32_MAX) return fail(MAPI_ERR_ARG, "matrix dimension exceeds 2^31-1");
  if (square && A->n_rows != A->n_cols) return fail(MAPI_ERR_ARG, "matrix must be square for a solve");
  const int64_t es = elem_size(A->dtype);
  if (!es) return fail(MAPI_ERR_ARG, "unknown dtype %d", A->dtype);
  if (A->ld < A->n_cols) return fail(MAPI_ERR_ARG, "ld (%lld) < n_cols (%lld)", (long long)A->ld, (long long)A->n_cols);
  if (!aligned16(A->data) || (A->ld * es) % 16 != 0)
    return fail(MAPI_ERR_ARG, "matrix base and row pitch must be 16-byte aligned");
  if (A->dtype == MAPI_FP8_E4M3 && !A->row_scale) return fail(MAPI_ERR_ARG, "FP8 storage needs row_scale");
  return MAPI_OK;
}

mapi_status check_opts(const mapi_opts* o) {
  if (!o) return fail(MAPI_ERR_ARG, "opts is NULL");
  if (o->max_iters < 0) return fail(MAPI_ERR_ARG, "max_iters < 0");
  if (!(o->tol >= 0.0)) return fail(MAPI_ERR_ARG, "tol must be >= 0");
  if (o->check_every < 0 || o->stall_iters < 0) return fail(MAPI_ERR_ARG, "check_every and stall_iters must be >= 0");
  return MAPI_OK;
}

DenseArgs dense_args(const mapi_dense* A) {
  return DenseArgs{A->data, A->ld, A->n_rows, A->n_cols, A->dtype, A->row_scale};
}

int ceil_log2(int64_t x) {
  int k = 0;
  while ((int64_t(1) << k) < x) ++k;
  return k;
}

std::tuple<int, int, int> bucket(int dtype, int64_t rows, int64_t cols) {
  return std::make_tuple(dtype, ceil_log2(rows), ceil_log2(cols));
}

DenseTuning tuning_for(mapi_ctx* c, const DenseArgs& a) {
  DenseTuning t = dense_default_tuning(a, c->cu_count, c->max_lds);
  auto it = c->tuned.find(bucket(a.dtype, a.n_rows, a.n_cols));
  if (it != c->tuned.end()) {
    t = it->second;
    if ((int64_t)dense_lds_bytes(a.dtype, a.n_cols, t.w_in_lds) + 1024 > c->max_lds) t.w_in_lds = 0;   // bucket spans sizes past the LDS
  }
  return t;
}

mapi_status to_dense_tuning(const mapi_tuning* u, DenseTuning* t) {
  if (!u) return fail(MAPI_ERR_ARG, "tuning is NULL");
  const int rw = u->rows_per_wave;
  if (!(rw == 1 || rw == 2 || rw == 4 || rw == 8)) return fail(MAPI_ERR_ARG, "rows_per_wave must be 1, 2, 4 or 8");
  if (u->waves != 4 && u->waves != 8) return fail(MAPI_ERR_ARG, "waves must be 4 or 8");
  if (u->blocks_per_cu < 1 || u->blocks_per_cu > 16) return fail(MAPI_ERR_ARG, "blocks_per_cu must be in 1..16");
  if (u->unroll != 2 && u->unroll != 4) return fail(MAPI_ERR_ARG, "unroll must be 2 or 4");
  t->rows_per_wave = rw;
  t->waves = u->waves;
  t->blocks = 0;
  t->blocks_per_cu = u->blocks_per_cu;
  t->unroll = u->unroll;
  if (u->w_in_lds < 0 || u->w_in_lds > 2) return fail(MAPI_ERR_ARG, "w_in_lds must be 0, 1 or 2");
  t->w_in_lds = u->w_in_lds;
  t->nontemporal = u->nontemporal ? 1 : 0;
  return MAPI_OK;
}

void from_dense_tuning(const DenseTuning& t, int cu_count, mapi_tuning* u) {
  u->rows_per_wave = t.rows_per_wave;
  u->waves = t.waves;
  u->blocks_per_cu = t.blocks_per_cu > 0 ? t.blocks_per_cu : (t.blocks > 0 ? (t.blocks + cu_count - 1) / cu_count : 0);
  u->unroll = t.unroll;
  u->w_in_lds = t.w_in_lds;
  u->nontemporal = t.nontemporal;
}

void load_tune_cache(mapi_ctx* c) {
  const char* path = std::getenv("MAPI_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  int dt, rb, cb, rw, wv, bpc, un, lds, nt;
  while (std::fscanf(f, "%d %d %d %d %d %d %d %d %d", &dt, &rb, &cb, &rw, &wv, &bpc, &un, &lds, &nt) == 9) {
    mapi_tuning u{rw, wv, bpc, un, lds, nt};
    DenseTuning t;
    if (to_dense_tuning(&u, &t) == MAPI_OK && lds_mode_ok(dt, t.w_in_lds)) c->tuned[std::make_tuple(dt, rb, cb)] = t;
  }
  std::fclose(f);
  g_err.clear();
}

void save_tune_entry(const std::tuple<int, int, int>& k, const DenseTuning& t) {
  const char* path = std::getenv("MAPI_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%d %d %d %d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k), t.rows_per_wave,
               t.waves, t.blocks_per_cu, t.unroll, t.w_in_lds, t.nontemporal);
  std::fclose(f);
}

void fill_info(mapi_info* info, const SolveState& s) {
  if (!info) return;
  info->iters = s.iter;
  info->converged = s.converged;
  info->residual = s.r;
  info->norm = s.nu;
  info->status = s.status;
}

}  // namespace

namespace mapi {

// Upper bound of the dense product kernel's block (partial) count for n rows: blocks
// of at least 4 waves of at least one row each, at most 16 blocks per compute unit.
int dense_part_bound(int64_t n, int cu_count) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + 3) / 4, (int64_t)cu_count * 16));
}

// Buffers of one dense solve, carved from one device region: the solve state, two sets
// of product and residual partials, the normalisation partials, two iterates and two
// products (a product that forms the previous iterate reads the other set).
struct DenseBufs {
  SolveState* st;
  double* pp[2];
  double* rp[2];
  double* part;
  float* wb[2];
  float* yb[2];
};

// Bytes of that region for an n x n system (the layout does not depend on the launch
// shape); with `base`, the buffers' addresses.
size_t dense_layout(int64_t n, int cu_count, char* base, DenseBufs* b) {
  const int P = dense_part_bound(n, cu_count);
  const int F = finalize_blocks(n);
  Layout L;
  const size_t o_st = L.take(sizeof(SolveState));
  const size_t o_pp = L.take(sizeof(double) * 2 * (size_t)P);
  const size_t o_rp = L.take(sizeof(double) * 2 * (size_t)P);
  const size_t o_part = L.take(sizeof(double) * 3 * (size_t)F);
  const size_t o_w0 = L.take(sizeof(float) * n);
  const size_t o_w1 = L.take(sizeof(float) * n);
  const size_t o_y0 = L.take(sizeof(float) * n);
  const size_t o_y1 = L.take(sizeof(float) * n);
  if (base && b) {
    b->st = reinterpret_cast<SolveState*>(base + o_st);
    b->pp[0] = reinterpret_cast<double*>(base + o_pp);
    b->pp[1] = b->pp[0] + P;
    b->rp[0] = reinterpret_cast<double*>(base + o_rp);
    b->rp[1] = b->rp[0] + P;
    b->part = reinterpret_cast<double*>(base + o_part);
    b->wb[0] = reinterpret_cast<float*>(base + o_w0);
    b->wb[1] = reinterpret_cast<float*>(base + o_w1);
    b->yb[0] = reinterpret_cast<float*>(base + o_y0);
    b->yb[1] = reinterpret_cast<float*>(base + o_y1);
  }
  return L.off;
}

size_t dense_ws_bytes(int64_t n, int cu_count) { return dense_layout(n, cu_count, nullptr, nullptr); }

mapi_status check_solve_args(const mapi_dense* A, const float* w0, const float* w_out, const mapi_opts* o, bool rpi) {
  mapi_status s;
  if ((s = check_dense(A, true)) != MAPI_OK) return s;
  if ((s = check_opts(o)) != MAPI_OK) return s;
  if (!w0 || !w_out) return fail(MAPI_ERR_ARG, "w0 and w_out must be device pointers");
  const int op = rpi ? MAPI_OP_DOT : o->op;
  if (op < MAPI_OP_MIN1 || op > MAPI_OP_DOT || (!rpi && op == MAPI_OP_DOT))
    return fail(MAPI_ERR_ARG, "op %d is not a MAPI product", o->op);
  return MAPI_OK;
}

// Iteration `it` of a dense solve, enqueued: the product of w_it (which, with w staged in
// LDS, the product forms itself from the previous y and partials: FusedPrev) and, without
// LDS staging, the normalisation launch.  With c->alternate, odd iterations sweep the
// rows in mirrored order, so each product starts on the rows the previous one read last,
// which the memory-side cache may still hold.  timed: record the launches in the
// context's kernel timing.
hipError_t enqueue_dense_iteration(mapi_ctx* c, const DenseArgs& da, int op, int norm, const DenseTuning& t, int P,
                                   const DenseBufs& B, int it, bool timed) {
  const bool fused = t.w_in_lds != 0;
  const int b = fused ? (it & 1) : 0;   // y and partials alternate when a product reads the previous ones
  {
    DenseArgs dl = da;
    dl.reverse = c->alternate ? (it & 1) : 0;
    TimedLaunch tm(c, MAPI_K_MAVP, timed ? &dl : nullptr);
    const FusedPrev fp{B.yb[b ^ 1], B.pp[b ^ 1], P, B.wb[it & 1], it, B.wb[(it & 1) ^ 1],
                       it >= 2 ? B.rp[b ^ 1] : nullptr, B.rp[b]};
    hipError_t e = launch_mavp_dense(dl, op, B.wb[it & 1], B.yb[b], B.pp[b], B.st, norm, t, c->cu_count, c->stream,
                                     (fused && it > 0) ? &fp : nullptr);
    if (e != hipSuccess) return e;
  }
  if (!fused) {
    Timed tm(c, MAPI_K_FINALIZE, timed);
    return launch_finalize(0, B.yb[0], B.wb[it & 1], B.wb[(it & 1) ^ 1], da.n_rows, B.st, B.pp[0], P, norm, B.part,
                           nullptr, 0.0, 0.0, c->stream);
  }
  return hipSuccess;
}

// Power iteration on a dense square matrix: MAPI (op, l1) or RPI (dot, l2).  Arguments
// checked by check_solve_args; ws: device region of dense_ws_bytes(n) bytes.
mapi_status run_dense(mapi_ctx* c, const mapi_dense* A, const float* w0, float* w_out, const mapi_opts* o,
                      mapi_info* info, bool rpi, char* ws) {
  mapi_status s;
  const int op = rpi ? MAPI_OP_DOT : o->op;
  const int64_t n = A->n_rows;
  const int norm = rpi ? NORM_L2 : NORM_L1;
  DenseBufs B;
  dense_layout(n, c->cu_count, ws, &B);
  SolveState* st = B.st;
  if (A->dtype == MAPI_F32 && small_solve_fits(n, op) && o->max_iters <= kSmallMaxIters &&
      !c->pinned.count(bucket(A->dtype, n, A->n_cols))) {
    // the whole solve in one launch: latency, not bandwidth, bounds this size (at most
    // kSmallMaxIters iterations, a fraction of a second, stay inside one kernel)
    HIP_TRY(launch_state_init(st, o->max_iters, o->tol, o->stall_iters, c->stream));
    {
      Timed tm(c, MAPI_K_MAVP);
      HIP_TRY(launch_solve_small(op, static_cast<const float*>(A->data), A->ld, n, w0, w_out, st, norm, o->final_l2,
                                 c->stream));
    }
    if ((s = sync_and_state(c, st)) != MAPI_OK) return s;
    fill_info(info, *c->st_host);
    if (c->st_host->status == MAPI_ERR_DEGENERATE)
      return fail(MAPI_ERR_DEGENERATE, "normaliser was zero or not finite after %d iterations", c->st_host->iter);
    return MAPI_OK;
  }
  const DenseArgs da = dense_args(A);
  const DenseTuning t = tuning_for(c, da);
  const int P = dense_part_count(da, t, c->cu_count);
  if (P > dense_part_bound(n, c->cu_count)) return fail(MAPI_ERR_ARG, "launch shape exceeds the partial bound");
  // With w staged in LDS, each product forms its own iterate from the previous y and
  // partials (FusedPrev), adds its share of the residual ||w_t - w_{t-1}||_1 to a
  // per-block partial, and advances the stop rule for the previous iteration: one
  // launch per iteration, the stop decision one launch late.  The last iteration is
  // normalised by the normalisation kernel.  Same arithmetic as the kernel pair.
  const bool fused = t.w_in_lds != 0;
  double* const* pp = B.pp;
  double* const* rp = B.rp;
  double* part = B.part;
  float* const* wb = B.wb;
  float* const* yb = B.yb;

  HIP_TRY(hipMemcpyAsync(wb[0], w0, sizeof(float) * n, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(launch_state_init(st, o->max_iters, o->tol, o->stall_iters, c->stream));
  if (c->dcheck_selftest) HIP_TRY(launch_dcheck_selftest(st, c->stream));
  const int check = o->check_every > 0 ? o->check_every : 16;
  int launched = 0;
  for (int it = 0; it < o->max_iters; ++it) {
    HIP_TRY(enqueue_dense_iteration(c, da, op, norm, t, P, B, it, true));
    launched = it + 1;
    if ((it + 1) % check == 0 && it + 1 < o->max_iters) {
      if ((s = sync_and_state(c, st)) != MAPI_OK) return s;
      if (c->st_host->done) break;
    }
  }
  if (fused && launched > 0) {
    // the last iteration's normalisation, after the stop rule for the one before it
    // (whose residual the last product formed)
    const int it = launched - 1;
    Timed tm(c, MAPI_K_FINALIZE);
    HIP_TRY(launch_finalize(0, yb[it & 1], wb[it & 1], wb[(it & 1) ^ 1], n, st, pp[it & 1], P, norm, part, nullptr,
                            0.0, 0.0, c->stream, it >= 1 ? rp[it & 1] : nullptr, P));
  }
  HIP_TRY(launch_finish(wb[0], wb[1], w_out, n, st, o->final_l2, c->stream, part));
  if ((s = sync_and_state(c, st)) != MAPI_OK) return s;
  fill_info(info, *c->st_host);
  if (c->st_host->status == MAPI_ERR_DEGENERATE)
    return fail(MAPI_ERR_DEGENERATE, "normaliser was zero or not finite after %d iterations", c->st_host->iter);
  return MAPI_OK;
}

size_t hybrid_ws_bytes(int64_t n, int cu_count) {
  return align_up(sizeof(float) * (size_t)n) + dense_ws_bytes(n, cu_count);
}

// Largest float64 partial-tile store of the Gram build over the products it runs with.
size_t gram_ws_max(int64_t D, int64_t N) {
  return std::max(gram_workspace_bytes(D, N, MAPI_OP_MIN1), gram_workspace_bytes(D, N, MAPI_OP_DOT));
}

// Region of mapi_pca_topk: the built and deflated matrices, the deflation partials, the
// current vector, the Gram build's partial tiles and a dense solve's buffers, then the
// float64 basis P and its products Q = A P (D x k each) last, so that the size grows by
// exactly 16 D bytes per vector.
struct PcaLayout {
  int64_t ldA;
  size_t o_A, o_Ai, o_qp, o_w, o_g, o_d, o_PQ, total;
};
PcaLayout pca_layout(int64_t D, int64_t k, size_t gram_bytes, int cu_count) {
  PcaLayout p;
  p.ldA = (D + 3) / 4 * 4;
  Layout L;
  p.o_A = L.take(sizeof(float) * D * p.ldA);
  p.o_Ai = L.take(sizeof(float) * D * p.ldA);
  p.o_qp = L.take(sizeof(double) * D * deflate_qpart_count());
  p.o_w = L.take(sizeof(float) * D);
  p.o_g = L.take(gram_bytes);
  p.o_d = L.take(dense_ws_bytes(D, cu_count));
  p.o_PQ = L.off;
  p.total = p.o_PQ + 2 * sizeof(double) * (size_t)D * (size_t)k;
  return p;
}

// Region of mapi_image_reconstruct (P pixels, N images).
struct ImageLayout {
  int64_t ldA, ldc;
  int G;
  size_t o_C, o_C2, o_Vc, o_m, o_perm, o_sums, o_P, o_Q, o_qp, o_pf, o_g, o_d, total;
};
ImageLayout image_layout(int64_t P, int64_t N, size_t gram_bytes, int cu_count) {
  ImageLayout l;
  l.ldA = (P + 3) / 4 * 4;     // 16-byte rows for the product kernel
  l.ldc = (N + 3) / 4 * 4;     // centred images, 16-byte rows for the Gram kernel
  l.G = (int)std::min<int64_t>(64, P);
  Layout L;
  l.o_C = L.take(sizeof(float) * P * l.ldA);
  l.o_C2 = L.take(sizeof(float) * P * l.ldA);
  l.o_Vc = L.take(sizeof(float) * P * l.ldc);
  l.o_m = L.take(sizeof(float) * P);
  l.o_perm = L.take(sizeof(int32_t) * P);
  l.o_sums = L.take(sizeof(double) * image_defl_sums_per_column() * (size_t)l.G * P);
  l.o_P = L.take(sizeof(double) * P);
  l.o_Q = L.take(sizeof(double) * P);
  l.o_qp = L.take(sizeof(double) * P * deflate_qpart_count());
  l.o_pf = L.take(sizeof(float) * P);
  l.o_g = L.take(gram_bytes);
  l.o_d = L.take(dense_ws_bytes(P, cu_count));
  l.total = L.off;
  return l;
}

// Whether a PageRank solve on n nodes with nnz links uses the column-split product.
bool pagerank_split(const mapi_ctx* c, int64_t n, int64_t nnz) {
  return c->csr_split_min_n > 0 && n >= c->csr_split_min_n && nnz > 0;
}

// Region of a PageRank solve with iterate type of `es` bytes, then the column-split
// copy of the link matrix when the solve uses it.
struct PrLayout {
  int PP, P;
  size_t o_st, o_pp, o_part, o_w0, o_w1, o_y, o_d, o_err, o_split, total;
};
PrLayout pagerank_layout(int64_t n, int64_t nnz, size_t es, bool split) {
  PrLayout l;
  const int F = finalize_blocks(n);
  l.PP = std::max(csr_part_count(n), split_combine_blocks(n));
  l.P = std::max(3 * F, 2 * pr_scalar_blocks(n));
  Layout L;
  l.o_st = L.take(sizeof(SolveState));
  l.o_pp = L.take(sizeof(double) * l.PP);
  l.o_part = L.take(sizeof(double) * l.P);
  l.o_w0 = L.take(es * n);
  l.o_w1 = L.take(es * n);
  l.o_y = L.take(es * n);
  l.o_d = L.take(n);
  l.o_err = L.take(sizeof(int32_t));
  l.o_split = L.take(split ? split_csr_bytes(n, nnz, es) : 0);
  l.total = L.off;
  return l;
}

// Region of mapi_minibatch: per-run records, the index-error flag, then the batch
// matrices of `range` steps of t and the runs' states.
size_t minibatch_bytes(int D, int range, int runs) {
  Layout L;
  L.take(sizeof(MbRun) * (size_t)runs);
  L.take(sizeof(int32_t));
  return L.off + minibatch_workspace_bytes(D, range, runs);
}

// Scratch of the single-product calls (mapi_mavp's aligned copy of w, the autotuner's
// w and y, mapi_read_reference's sink).
size_t product_ws_bytes(int64_t n_rows, int64_t n_cols) {
  return align_up(sizeof(float) * (size_t)n_cols) + align_up(sizeof(float) * (size_t)n_rows);
}

// The autotuner's: that scratch and, for a square matrix, a dense solve's buffers (its
// trials run solve iterations).
size_t autotune_ws_bytes(int64_t n_rows, int64_t n_cols, int cu_count) {
  return product_ws_bytes(n_rows, n_cols) + (n_rows == n_cols ? dense_ws_bytes(n_rows, cu_count) : 0);
}

// Region of mapi_factored_solve: a dense solve's buffers for the D rows of X, then the
// column product's chunk partials (RC x N floats) and z (N floats).
struct FactLayout {
  size_t o_d, o_zp, o_z, total;
};
FactLayout factored_layout(int64_t D, int64_t N, int cu_count) {
  FactLayout f;
  Layout L;
  f.o_d = L.take(dense_ws_bytes(D, cu_count));
  f.o_zp = L.take(sizeof(float) * (size_t)col_product_chunks(D) * (size_t)N);
  f.o_z = L.take(sizeof(float) * (size_t)N);
  f.total = L.off;
  return f;
}

// mapi_solve / rpi_solve: checks, then the solve in the context's (or the caller's) workspace.
mapi_status solve_entry(mapi_ctx* c, const mapi_dense* A, const float* w0, float* w_out, const mapi_opts* o,
                        mapi_info* info, bool rpi) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  mapi_status s;
  if ((s = check_solve_args(A, w0, w_out, o, rpi)) != MAPI_OK) return s;
  HIP_TRY(hipSetDevice(c->device));
  char* ws = nullptr;
  if ((s = acquire(c, &c->ws, &c->ws_bytes, dense_ws_bytes(A->n_rows, c->cu_count), &ws)) != MAPI_OK) return s;
  return run_dense(c, A, w0, w_out, o, info, rpi, ws);
}

}  // namespace mapi

namespace {

// PageRank power iteration with a float32 or float64 iterate T (eq. 11 split sums).
template <typename T>
mapi_status pagerank_run(mapi_ctx* c, const mapi_csr* H, double alpha, int32_t method, const T* w0, T* w_out,
                         const mapi_opts* o, mapi_info* info) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  if (!H || !H->row_ptr || !w_out) return fail(MAPI_ERR_ARG, "H, H->row_ptr and w_out are required");
  if (H->n <= 0 || H->n > INT32_MAX || H->nnz < 0 || H->nnz > INT32_MAX) return fail(MAPI_ERR_ARG, "bad n or nnz");
  if (H->nnz > 0 && (!H->col || !H->val)) return fail(MAPI_ERR_ARG, "col and val are required when nnz > 0");
  if (!(alpha > 0.0 && alpha < 1.0)) return fail(MAPI_ERR_ARG, "alpha must be in (0, 1)");
  if (method != MAPI_METHOD_MAPI && method != MAPI_METHOD_RPI) return fail(MAPI_ERR_ARG, "method %d", method);
  mapi_status s;
  if ((s = check_opts(o)) != MAPI_OK) return s;
  HIP_TRY(hipSetDevice(c->device));
  const int64_t n = H->n;
  bool split = pagerank_split(c, n, H->nnz);
  const PrLayout l = pagerank_layout(n, H->nnz, sizeof(T), split);
  char* base = nullptr;
  if ((s = acquire(c, &c->ws, &c->ws_bytes, l.total, &base)) != MAPI_OK) return s;
  SolveState* st = reinterpret_cast<SolveState*>(base + l.o_st);
  double* pprod = reinterpret_cast<double*>(base + l.o_pp);
  double* part = reinterpret_cast<double*>(base + l.o_part);
  T* wb[2] = {reinterpret_cast<T*>(base + l.o_w0), reinterpret_cast<T*>(base + l.o_w1)};
  T* y = reinterpret_cast<T*>(base + l.o_y);
  uint8_t* dangling = reinterpret_cast<uint8_t*>(base + l.o_d);
  int32_t* err = reinterpret_cast<int32_t*>(base + l.o_err);

  HIP_TRY(hipMemsetAsync(err, 0, sizeof(int32_t), c->stream));
  HIP_TRY(launch_csr_prep(H->row_ptr, H->col, n, H->nnz, dangling, err, c->stream));
  int32_t err_h = 0;
  HIP_TRY(hipMemcpyAsync(&err_h, err, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (err_h) return fail(MAPI_ERR_ARG, "invalid CSR arrays (code %d)", err_h);
  // the column-split copy of the validated matrix, unless a row has too many links in
  // one block for its layout (then the plain product runs); built before the product of
  // iteration c->csr_split_after, if the solve gets that far
  SplitCsr sp;
  const int split_at = split ? c->csr_split_after : -1;
  split = false;
  auto build_split = [&]() -> mapi_status {
    sp = split_csr_place(base + l.o_split, n, H->nnz, sizeof(T));
    HIP_TRY(hipMemsetAsync(sp.flags, 0, sizeof(int32_t), c->stream));
    HIP_TRY(launch_split_count(H->row_ptr, H->col, H->val, sp, c->stream));
    int32_t flags_h = 0;
    HIP_TRY(hipMemcpyAsync(&flags_h, sp.flags, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (!flags_h) {
      HIP_TRY(launch_split_fill(H->row_ptr, H->col, H->val, sp, c->stream));
      split = true;
    }
    return MAPI_OK;
  };
  if (split_at == 0 && (s = build_split()) != MAPI_OK) return s;

  const double inv_n = 1.0 / (double)n;
  const double cc = (1.0 - alpha) * inv_n;
  if (w0) {
    HIP_TRY(hipMemcpyAsync(wb[0], w0, sizeof(T) * n, hipMemcpyDeviceToDevice, c->stream));
  } else if constexpr (sizeof(T) == 4) {
    HIP_TRY(launch_fill_f32(wb[0], n, (float)inv_n, c->stream));
  } else {
    HIP_TRY(launch_fill_f64(wb[0], n, inv_n, c->stream));
  }
  HIP_TRY(launch_state_init(st, o->max_iters, o->tol, o->stall_iters, c->stream));
  HIP_TRY(launch_pr_scalars<T>(method, wb[0], n, dangling, cc, inv_n, st, part, c->stream));
  const int check = o->check_every > 0 ? o->check_every : 16;
  const int mode = method == MAPI_METHOD_MAPI ? 1 : 2;
  for (int it = 0; it < o->max_iters; ++it) {
    T* wc = wb[it & 1];
    T* wn = wb[(it & 1) ^ 1];
    if (it > 0 && it == split_at) {   // still running: switch to the split product from here
      if ((s = sync_and_state(c, st)) != MAPI_OK) return s;
      if (c->st_host->done) break;
      if ((s = build_split()) != MAPI_OK) return s;
    }
    const int PP = split ? split_combine_blocks(n) : csr_part_count(n);
    {
      Timed tm(c, MAPI_K_CSR);
      if (split)
        HIP_TRY(launch_csr_split_product<T>(method, sp, wc, y, pprod, st, alpha, cc, inv_n, c->stream));
      else
        HIP_TRY(launch_csr_product<T>(method, H->row_ptr, H->col, H->val, n, wc, y, pprod, st, alpha, cc, inv_n,
                                      c->stream));
    }
    {
      Timed tm(c, MAPI_K_FINALIZE);
      if constexpr (sizeof(T) == 4)
        HIP_TRY(launch_finalize(mode, y, wc, wn, n, st, pprod, PP, NORM_L1, part, dangling, cc, inv_n, c->stream));
      else
        HIP_TRY(launch_finalize_f64(mode, y, wc, wn, n, st, pprod, PP, part, dangling, cc, inv_n, c->stream));
    }
    if ((it + 1) % check == 0 && it + 1 < o->max_iters) {
      if ((s = sync_and_state(c, st)) != MAPI_OK) return s;
      if (c->st_host->done) break;
    }
  }
  if constexpr (sizeof(T) == 4)
    HIP_TRY(launch_finish(wb[0], wb[1], w_out, n, st, o->final_l2, c->stream, part));
  else
    HIP_TRY(launch_finish_f64(wb[0], wb[1], w_out, n, st, o->final_l2, c->stream, part));
  if ((s = sync_and_state(c, st)) != MAPI_OK) return s;
  fill_info(info, *c->st_host);
  if (c->st_host->status == MAPI_ERR_DEGENERATE)
    return fail(MAPI_ERR_DEGENERATE, "normaliser was zero or not finite after %d iterations", c->st_host->iter);
  return MAPI_OK;
}

}  // namespace

// ====================================================================== C-ABI
extern "C" {

const char* mapi_last_error(void) { return g_err.c_str(); }
const char* mapi_version(void) { return "mapi-gfx950 0.1"; }

mapi_status mapi_create(int device, void* hip_stream, mapi_ctx** out) {
  if (!out) return fail(MAPI_ERR_ARG, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(MAPI_ERR_ARG, "device %d not present (%d devices)", device, ndev);
  HIP_TRY(hipSetDevice(device));
  mapi_ctx* c = new (std::nothrow) mapi_ctx();
  if (!c) return fail(MAPI_ERR_ALLOC, "context allocation failed");
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0) {
    c->cu_count = prop.multiProcessorCount;
    if (prop.sharedMemPerBlock > 0) c->max_lds = (int)prop.sharedMemPerBlock;
  }
  load_tune_cache(c);
  if (const char* e = std::getenv("MAPI_DENSE_ALTERNATE")) c->alternate = std::atoi(e) != 0;
  if (const char* e = std::getenv("MAPI_DCHECK_SELFTEST")) c->dcheck_selftest = std::atoi(e) != 0;
  mapi_status ss = scratch_setup(device, &c->scratch);
  if (ss != MAPI_OK) {
    delete c;
    return ss;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&c->st_host), sizeof(SolveState), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return fail(MAPI_ERR_ALLOC, "pinned host allocation failed");
  }
  *out = c;
  return MAPI_OK;
}

void mapi_destroy(mapi_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  collect_timing(c);
  for (auto e : c->pool) (void)hipEventDestroy(e);
  if (c->ws) (void)hipFree(c->ws);
  if (c->big) (void)hipFree(c->big);
  if (c->mid) (void)hipFree(c->mid);
  if (c->gws) (void)hipFree(c->gws);
  mapi_batch_release(c);
  if (c->st_host) (void)hipHostFree(c->st_host);
  delete c;
}

mapi_status mapi_set_stream(mapi_ctx* c, void* hip_stream) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->stream = static_cast<hipStream_t>(hip_stream);
  return MAPI_OK;
}

mapi_status mapi_workspace_size(const mapi_ctx* c, int32_t kind, int64_t n, int64_t nnz, size_t* bytes) {
  if (!c || !bytes) return fail(MAPI_ERR_ARG, "ctx and bytes are required");
  *bytes = 0;
  if (n <= 0 || n > INT32_MAX) return fail(MAPI_ERR_ARG, "n must be in [1, 2^31)");
  const int cu = c->cu_count;
  switch (kind) {
    case MAPI_WS_SOLVE: *bytes = dense_ws_bytes(n, cu); break;
    case MAPI_WS_HYBRID: *bytes = hybrid_ws_bytes(n, cu); break;
    case MAPI_WS_PAGERANK:
    case MAPI_WS_PAGERANK_F64:
      if (nnz < 0 || nnz > INT32_MAX) return fail(MAPI_ERR_ARG, "nnz (the link count) must be in [0, 2^31)");
      *bytes = pagerank_layout(n, nnz, kind == MAPI_WS_PAGERANK ? sizeof(float) : sizeof(double),
                               pagerank_split(c, n, nnz)).total;
      break;
    case MAPI_WS_PRODUCT:
      if (nnz <= 0) return fail(MAPI_ERR_ARG, "nnz (the column count) must be positive");
      *bytes = autotune_ws_bytes(n, nnz, cu);
      break;
    case MAPI_WS_MINGRAM:
      if (nnz <= 0) return fail(MAPI_ERR_ARG, "nnz (the sample count N) must be positive");
      *bytes = gram_ws_max(n, nnz);
      break;
    case MAPI_WS_PCA:
      if (nnz <= 0) return fail(MAPI_ERR_ARG, "nnz (the sample count N) must be positive");
      *bytes = pca_layout(n, 1, gram_ws_max(n, nnz), cu).total;
      break;
    case MAPI_WS_PCA_VECTOR: *bytes = 2 * sizeof(double) * (size_t)n; break;
    case MAPI_WS_IMAGE:
      if (nnz < 2) return fail(MAPI_ERR_ARG, "nnz (the image count N) must be at least 2");
      *bytes = image_layout(n, nnz, gram_ws_max(n, nnz), cu).total;
      break;
    case MAPI_WS_MINIBATCH:
      if (nnz <= 0 || nnz > INT32_MAX) return fail(MAPI_ERR_ARG, "nnz (the run count) must be positive");
      if (n > minibatch_max_d()) return fail(MAPI_ERR_UNSUPPORTED, "D > %d", minibatch_max_d());
      *bytes = minibatch_bytes((int)n, minibatch_range((int)n, INT32_MAX, (int)nnz), (int)nnz);
      break;
    case MAPI_WS_FACTORED:
      if (nnz <= 0 || nnz > INT32_MAX) return fail(MAPI_ERR_ARG, "nnz (the sample count N) must be positive");
      *bytes = factored_layout(n, nnz, cu).total;
      break;
    case MAPI_WS_MINIBATCH_MIN:
      if (nnz <= 0 || nnz > INT32_MAX) return fail(MAPI_ERR_ARG, "nnz (the run count) must be positive");
      if (n > minibatch_max_d()) return fail(MAPI_ERR_UNSUPPORTED, "D > %d", minibatch_max_d());
      *bytes = minibatch_bytes((int)n, 1, (int)nnz);
      break;
    default: return fail(MAPI_ERR_ARG, "unknown workspace kind %d", kind);
  }
  *bytes = align_up(*bytes);
  return MAPI_OK;
}

mapi_status mapi_set_workspace(mapi_ctx* c, void* dev_ptr, size_t bytes) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  if (dev_ptr && (reinterpret_cast<uintptr_t>(dev_ptr) & 255u) != 0)
    return fail(MAPI_ERR_ARG, "the workspace must be 256-byte aligned");
  if (dev_ptr && bytes == 0) return fail(MAPI_ERR_ARG, "a workspace needs a non-zero size");
  HIP_TRY(hipSetDevice(c->device));
  // the previous workspace (the caller's or the context's own) may still be read by
  // enqueued work; the context's own buffers are given back
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->side) HIP_TRY(hipStreamSynchronize(c->side));
  for (auto* own : {&c->ws, &c->big, &c->mid, &c->gws}) {
    if (*own) HIP_TRY(hipFree(*own));
    *own = nullptr;
  }
  c->ws_bytes = c->big_bytes = c->mid_bytes = c->gws_bytes = 0;
  mapi_batch_free_arena(c);
  c->user_ws = static_cast<char*>(dev_ptr);
  c->user_ws_bytes = dev_ptr ? bytes : 0;
  return MAPI_OK;
}

mapi_status mapi_pagerank_split_after(mapi_ctx* c, int32_t iters) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  if (iters < 0) return fail(MAPI_ERR_ARG, "iters must be >= 0");
  c->csr_split_after = iters;
  return MAPI_OK;
}

mapi_status mapi_pagerank_split_config(mapi_ctx* c, int64_t min_n) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  c->csr_split_min_n = min_n > 0 ? min_n : 0;
  return MAPI_OK;
}

mapi_status mapi_timing_enable(mapi_ctx* c, int enable) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  c->timing = enable != 0;
  return MAPI_OK;
}

mapi_status mapi_timing_get(mapi_ctx* c, int kind, double* total_ms, int64_t* launches) {
  if (!c || kind < 0 || kind >= MAPI_K_KINDS) return fail(MAPI_ERR_ARG, "bad context or kernel kind");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->stream));
  collect_timing(c);
  if (total_ms) *total_ms = c->t_ms[kind];
  if (launches) *launches = c->t_n[kind];
  return MAPI_OK;
}

mapi_status mapi_timing_reset(mapi_ctx* c) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->stream));
  collect_timing(c);
  for (int k = 0; k < MAPI_K_KINDS; ++k) {
    c->t_ms[k] = 0.0;
    c->t_n[k] = 0;
  }
  return MAPI_OK;
}

mapi_status mapi_mavp(mapi_ctx* c, const mapi_dense* A, const float* w, float* y, int32_t op) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  mapi_status s;
  if ((s = check_dense(A, false)) != MAPI_OK) return s;
  if (!w || !y) return fail(MAPI_ERR_ARG, "w and y must be device pointers");
  if (op < MAPI_OP_MIN1 || op > MAPI_OP_DOT) return fail(MAPI_ERR_ARG, "unknown op %d", op);
  HIP_TRY(hipSetDevice(c->device));
  const DenseArgs da = dense_args(A);
  const DenseTuning t = tuning_for(c, da);
  const float* wv = w;
  if (!aligned16(w)) {
    char* base = nullptr;
    if ((s = acquire(c, &c->ws, &c->ws_bytes, sizeof(float) * (size_t)A->n_cols, &base)) != MAPI_OK) return s;
    HIP_TRY(hipMemcpyAsync(base, w, sizeof(float) * A->n_cols, hipMemcpyDeviceToDevice, c->stream));
    wv = reinterpret_cast<const float*>(base);
  }
  {
    DenseArgs dl = da;
    TimedLaunch tm(c, MAPI_K_MAVP, &dl);
    HIP_TRY(launch_mavp_dense(dl, op, wv, y, nullptr, nullptr, NORM_NONE, t, c->cu_count, c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  collect_timing(c);
  return MAPI_OK;
}

static mapi_status time_product(mapi_ctx* c, const DenseArgs& da, int op, const float* w, float* y,
                                const DenseTuning& t, int reps, double* avg_ms) {
  hipEvent_t a = get_event(c), b = get_event(c);
  if (!a || !b) return fail(MAPI_ERR_HIP, "event creation failed");
  HIP_TRY(launch_mavp_dense(da, op, w, y, nullptr, nullptr, NORM_NONE, t, c->cu_count, c->stream));   // warm
  HIP_TRY(hipEventRecord(a, c->stream));
  for (int r = 0; r < reps; ++r)
    HIP_TRY(launch_mavp_dense(da, op, w, y, nullptr, nullptr, NORM_NONE, t, c->cu_count, c->stream));
  HIP_TRY(hipEventRecord(b, c->stream));
  HIP_TRY(hipEventSynchronize(b));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, a, b));
  c->pool.push_back(a);
  c->pool.push_back(b);
  *avg_ms = ms / reps;
  return MAPI_OK;
}

// Average time of one solve iteration in shape t (square matrices): `reps` iterations
// enqueued exactly as a solve enqueues them, after two untimed ones, on a state that never
// stops (tolerance 0, no stall rule).  ws: dense_ws_bytes(n) bytes.  *degenerate: the
// matrix gave a zero normaliser, so the launches returned early and the time means nothing.
static mapi_status time_iterations(mapi_ctx* c, const DenseArgs& da, int op, const float* w0, char* ws,
                                   const DenseTuning& t, int reps, double* avg_ms, bool* degenerate) {
  DenseBufs B;
  dense_layout(da.n_rows, c->cu_count, ws, &B);
  const int norm = op == MAPI_OP_DOT ? NORM_L2 : NORM_L1;
  const int P = dense_part_count(da, t, c->cu_count);
  hipEvent_t a = get_event(c), b = get_event(c);
  if (!a || !b) return fail(MAPI_ERR_HIP, "event creation failed");
  HIP_TRY(hipMemcpyAsync(B.wb[0], w0, sizeof(float) * da.n_rows, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(launch_state_init(B.st, reps + 8, 0.0, 0, c->stream));
  HIP_TRY(enqueue_dense_iteration(c, da, op, norm, t, P, B, 0, false));
  HIP_TRY(enqueue_dense_iteration(c, da, op, norm, t, P, B, 1, false));
  HIP_TRY(hipEventRecord(a, c->stream));
  for (int it = 2; it < reps + 2; ++it) HIP_TRY(enqueue_dense_iteration(c, da, op, norm, t, P, B, it, false));
  HIP_TRY(hipEventRecord(b, c->stream));
  mapi_status s;
  if ((s = sync_and_state(c, B.st)) != MAPI_OK) return s;
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, a, b));
  c->pool.push_back(a);
  c->pool.push_back(b);
  *avg_ms = ms / reps;
  *degenerate = c->st_host->done != 0;
  return MAPI_OK;
}

mapi_status mapi_mavp_timed(mapi_ctx* c, const mapi_dense* A, const float* w, float* y, int32_t op,
                            const mapi_tuning* tu, int32_t reps, double* avg_ms) {
  if (!c || !avg_ms) return fail(MAPI_ERR_ARG, "ctx or avg_ms is NULL");
  mapi_status s;
  if ((s = check_dense(A, false)) != MAPI_OK) return s;
  if (!w || !y || !aligned16(w)) return fail(MAPI_ERR_ARG, "w (16-byte aligned) and y must be device pointers");
  if (op < MAPI_OP_MIN1 || op > MAPI_OP_DOT) return fail(MAPI_ERR_ARG, "unknown op %d", op);
  if (reps < 1) return fail(MAPI_ERR_ARG, "reps must be >= 1");
  DenseTuning t;
  if ((s = to_dense_tuning(tu, &t)) != MAPI_OK) return s;
  const DenseArgs da = dense_args(A);
  if (!lds_mode_ok(da.dtype, t.w_in_lds)) return fail(MAPI_ERR_ARG, "w_in_lds 2 needs FP8 storage");
  if ((int64_t)dense_lds_bytes(da.dtype, da.n_cols, t.w_in_lds) + 1024 > c->max_lds) return fail(MAPI_ERR_ARG, "w does not fit in LDS");
  HIP_TRY(hipSetDevice(c->device));
  return time_product(c, da, op, w, y, t, reps, avg_ms);
}

mapi_status mapi_read_reference(mapi_ctx* c, const void* src, size_t bytes, int32_t reps, double* avg_ms) {
  if (!c || !src || !avg_ms) return fail(MAPI_ERR_ARG, "NULL argument");
  if (bytes == 0 || bytes % 16 != 0 || !aligned16(src))
    return fail(MAPI_ERR_ARG, "bytes must be a non-zero multiple of 16 and src 16-byte aligned");
  if (reps < 1) return fail(MAPI_ERR_ARG, "reps must be >= 1");
  HIP_TRY(hipSetDevice(c->device));
  mapi_status s;
  char* base = nullptr;
  if ((s = acquire(c, &c->ws, &c->ws_bytes, 256, &base)) != MAPI_OK) return s;
  uint32_t* sink = reinterpret_cast<uint32_t*>(base);
  hipEvent_t a = get_event(c), b = get_event(c);
  if (!a || !b) return fail(MAPI_ERR_HIP, "event creation failed");
  // the fastest of 12 launch shapes: 1..32 blocks of 256 threads per compute unit, four
  // or eight loads per lane in flight
  const int64_t n16 = (int64_t)(bytes / 16);
  double best = 1e30;
  for (int unroll : {4, 8})
    for (int bpc : {1, 2, 4, 8, 16, 32}) {
      const int blocks = c->cu_count * bpc;
      HIP_TRY(launch_read16(src, n16, sink, blocks, unroll, c->stream));
      HIP_TRY(hipEventRecord(a, c->stream));
      for (int r = 0; r < reps; ++r) HIP_TRY(launch_read16(src, n16, sink, blocks, unroll, c->stream));
      HIP_TRY(hipEventRecord(b, c->stream));
      HIP_TRY(hipEventSynchronize(b));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, a, b));
      best = std::min(best, (double)ms / reps);
    }
  c->pool.push_back(a);
  c->pool.push_back(b);
  *avg_ms = best;
  return MAPI_OK;
}

mapi_status mapi_autotune_dense(mapi_ctx* c, const mapi_dense* A, int32_t op, int32_t reps, mapi_tuning* best,
                                double* best_ms) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  mapi_status s;
  if ((s = check_dense(A, false)) != MAPI_OK) return s;
  if (op < MAPI_OP_MIN1 || op > MAPI_OP_DOT) return fail(MAPI_ERR_ARG, "unknown op %d", op);
  if (reps < 1) reps = 3;
  HIP_TRY(hipSetDevice(c->device));
  const DenseArgs da = dense_args(A);
  char* base = nullptr;
  if ((s = acquire(c, &c->ws, &c->ws_bytes, autotune_ws_bytes(da.n_rows, da.n_cols, c->cu_count), &base)) != MAPI_OK)
    return s;
  float* w = reinterpret_cast<float*>(base);
  float* y = reinterpret_cast<float*>(base + align_up(sizeof(float) * (size_t)da.n_cols));
  char* dws = base + product_ws_bytes(da.n_rows, da.n_cols);
  HIP_TRY(launch_fill_f32(w, da.n_cols, 1.0f / (float)da.n_cols, c->stream));
  DenseTuning bt = dense_default_tuning(da, c->cu_count, c->max_lds);
  double bms = 1e30;
  DenseTuning bl = bt;      // fastest shape that stages w in LDS
  double blms = 1e30;
  // A square matrix is tuned on solve iterations (the product as a solve launches it,
  // with the iterate formed inside it or by the normalisation launch, in the solve's
  // sweep order), unless its normaliser is zero; a rectangular one on plain products.
  bool iterate = da.n_rows == da.n_cols;
  std::vector<std::pair<double, DenseTuning>> timed;   // every candidate's first timing
  for (int rw : {1, 2, 4, 8}) {
    if (rw > 1 && rw > da.n_rows) continue;
    for (int waves : {4, 8})
      for (int bpc : {1, 2, 4, 8})
        for (int un : {2, 4})
          for (int lds = 0; lds <= 2; ++lds)
            for (int nt = 0; nt <= 1; ++nt) {
              if (!lds_mode_ok(da.dtype, lds) ||
                  (int64_t)dense_lds_bytes(da.dtype, da.n_cols, lds) + 1024 > c->max_lds)
                continue;
              DenseTuning t{rw, waves, 0, lds, bpc, un, nt};
              double ms = 0.0;
              bool degenerate = false;
              if (iterate && (s = time_iterations(c, da, op, w, dws, t, reps, &ms, &degenerate)) != MAPI_OK) return s;
              if (degenerate) {   // start over on plain products
                iterate = false;
                bms = blms = 1e30;
                bt = bl = dense_default_tuning(da, c->cu_count, c->max_lds);
                timed.clear();
              }
              if (!iterate && (s = time_product(c, da, op, w, y, t, reps, &ms)) != MAPI_OK) return s;
              timed.emplace_back(ms, t);
              if (ms < bms) {
                bms = ms;
                bt = t;
              }
              if (lds != 0 && ms < blms) {
                blms = ms;
                bl = t;
              }
            }
  }
  // Solve iterations: the shapes within a few percent of each other are ranked by the
  // noise of one timing, so the six fastest are timed three more times, in turn (a slow
  // spell of the device then hits all of them), and the best of each one's four timings
  // decides.
  if (iterate && timed.size() > 1) {
    std::sort(timed.begin(), timed.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    const size_t top = std::min<size_t>(6, timed.size());
    for (int round = 0; round < 3; ++round)
      for (size_t i = 0; i < top; ++i) {
        double ms = 0.0;
        bool degenerate = false;
        if ((s = time_iterations(c, da, op, w, dws, timed[i].second, reps, &ms, &degenerate)) != MAPI_OK) return s;
        timed[i].first = std::min(timed[i].first, ms);
      }
    size_t bi = 0;
    for (size_t i = 1; i < top; ++i)
      if (timed[i].first < timed[bi].first) bi = i;
    bt = timed[bi].second;
    bms = timed[bi].first;
  }
  // On plain products, shapes that stage w in LDS are kept when within 3 % of the
  // fastest: in a solve they form each iterate inside the next product (no normalisation
  // launch, several microseconds an iteration).
  if (!iterate && bt.w_in_lds == 0 && blms <= 1.03 * bms) {
    bt = bl;
    bms = blms;
  }
  const auto key = bucket(da.dtype, da.n_rows, da.n_cols);
  c->tuned[key] = bt;
  save_tune_entry(key, bt);
  if (best) from_dense_tuning(bt, c->cu_count, best);
  if (best_ms) *best_ms = bms;
  return MAPI_OK;
}

mapi_status mapi_tuning_get(mapi_ctx* c, int32_t dtype, int64_t n_rows, int64_t n_cols, mapi_tuning* out) {
  if (!c || !out) return fail(MAPI_ERR_ARG, "ctx or out is NULL");
  if (n_rows <= 0 || n_cols <= 0 || elem_size(dtype) == 0) return fail(MAPI_ERR_ARG, "bad bucket");
  DenseArgs da{nullptr, n_cols, n_rows, n_cols, dtype, nullptr};
  from_dense_tuning(tuning_for(c, da), c->cu_count, out);
  return MAPI_OK;
}

mapi_status mapi_tuning_set(mapi_ctx* c, int32_t dtype, int64_t n_rows, int64_t n_cols, const mapi_tuning* tu) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  if (n_rows <= 0 || n_cols <= 0 || elem_size(dtype) == 0) return fail(MAPI_ERR_ARG, "bad bucket");
  DenseTuning t;
  mapi_status s;
  if ((s = to_dense_tuning(tu, &t)) != MAPI_OK) return s;
  if (!lds_mode_ok(dtype, t.w_in_lds)) return fail(MAPI_ERR_ARG, "w_in_lds 2 needs FP8 storage");
  c->tuned[bucket(dtype, n_rows, n_cols)] = t;
  c->pinned.insert(bucket(dtype, n_rows, n_cols));
  return MAPI_OK;
}

mapi_status mapi_copy_reference(mapi_ctx* c, const void* src, void* dst, size_t bytes, int32_t reps,
                                double* avg_ms) {
  if (!c || !src || !dst || !avg_ms) return fail(MAPI_ERR_ARG, "NULL argument");
  if (bytes == 0 || bytes % 16 != 0 || !aligned16(src) || !aligned16(dst))
    return fail(MAPI_ERR_ARG, "bytes must be a non-zero multiple of 16 and buffers 16-byte aligned");
  if (reps < 1) return fail(MAPI_ERR_ARG, "reps must be >= 1");
  HIP_TRY(hipSetDevice(c->device));
  hipEvent_t a = get_event(c), b = get_event(c);
  if (!a || !b) return fail(MAPI_ERR_HIP, "event creation failed");
  HIP_TRY(launch_copy16(src, dst, bytes / 16, c->cu_count, c->stream));
  HIP_TRY(hipEventRecord(a, c->stream));
  for (int r = 0; r < reps; ++r) HIP_TRY(launch_copy16(src, dst, bytes / 16, c->cu_count, c->stream));
  HIP_TRY(hipEventRecord(b, c->stream));
  HIP_TRY(hipEventSynchronize(b));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, a, b));
  c->pool.push_back(a);
  c->pool.push_back(b);
  *avg_ms = ms / reps;
  return MAPI_OK;
}

mapi_status mapi_solve(mapi_ctx* c, const mapi_dense* A, const float* w0, float* w_out, const mapi_opts* opts,
                       mapi_info* info) {
  return solve_entry(c, A, w0, w_out, opts, info, false);
}

mapi_status rpi_solve(mapi_ctx* c, const mapi_dense* A, const float* w0, float* w_out, const mapi_opts* opts,
                      mapi_info* info) {
  return solve_entry(c, A, w0, w_out, opts, info, true);
}

mapi_status mapi_hybrid_solve(mapi_ctx* c, const mapi_dense* A, const float* w0, float* w_out,
                              const mapi_opts* mapi_o, const mapi_opts* rpi_o, mapi_info* info_mapi,
                              mapi_info* info_rpi) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  mapi_status s;
  if ((s = check_solve_args(A, w0, w_out, mapi_o, false)) != MAPI_OK) return s;
  if ((s = check_opts(rpi_o)) != MAPI_OK) return s;
  HIP_TRY(hipSetDevice(c->device));
  char* base = nullptr;
  if ((s = acquire(c, &c->mid, &c->mid_bytes, hybrid_ws_bytes(A->n_rows, c->cu_count), &base)) != MAPI_OK) return s;
  float* mid = reinterpret_cast<float*>(base);
  char* ws = base + align_up(sizeof(float) * (size_t)A->n_rows);
  mapi_opts o1 = *mapi_o;
  o1.final_l2 = 1;     // the hand-over vector has unit l2 norm
  if ((s = run_dense(c, A, w0, mid, &o1, info_mapi, false, ws)) != MAPI_OK) return s;
  return run_dense(c, A, mid, w_out, rpi_o, info_rpi, true, ws);
}

mapi_status mapi_factored_solve(mapi_ctx* c, const float* X, int64_t D, int64_t N, int64_t ldx, double scale,
                                const float* w0, float* w_out, const mapi_opts* o, mapi_info* info) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  if (!X || !w0 || !w_out) return fail(MAPI_ERR_ARG, "X, w0 and w_out must be device pointers");
  if (D <= 0 || N <= 0 || ldx < N || D > INT32_MAX || N > INT32_MAX) return fail(MAPI_ERR_ARG, "bad shape");
  if (!aligned16(X) || ldx % 4 != 0) return fail(MAPI_ERR_ARG, "X base and row pitch must be 16-byte aligned");
  if (!(scale > 0.0) || !(scale < INFINITY)) return fail(MAPI_ERR_ARG, "scale must be positive and finite");
  mapi_status s;
  if ((s = check_opts(o)) != MAPI_OK) return s;
  if (o->op != MAPI_OP_MIN1 && o->op != MAPI_OP_MIN2)
    return fail(MAPI_ERR_UNSUPPORTED, "the factored operator is built for the min1 and min2 products");
  HIP_TRY(hipSetDevice(c->device));
  const FactLayout fl = factored_layout(D, N, c->cu_count);
  char* base = nullptr;
  if ((s = acquire(c, &c->ws, &c->ws_bytes, fl.total, &base)) != MAPI_OK) return s;
  DenseBufs B;
  dense_layout(D, c->cu_count, base + fl.o_d, &B);
  float* zpart = reinterpret_cast<float*>(base + fl.o_zp);
  float* z = reinterpret_cast<float*>(base + fl.o_z);
  const DenseArgs da{X, ldx, D, N, MAPI_F32, nullptr};
  const DenseTuning t = tuning_for(c, da);
  const int P = dense_part_count(da, t, c->cu_count);
  if (P > dense_part_bound(D, c->cu_count)) return fail(MAPI_ERR_ARG, "launch shape exceeds the partial bound");
  SolveState* st = B.st;
  HIP_TRY(hipMemcpyAsync(B.wb[0], w0, sizeof(float) * D, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(launch_state_init(st, o->max_iters, o->tol, o->stall_iters, c->stream));
  const int check = o->check_every > 0 ? o->check_every : 16;
  for (int it = 0; it < o->max_iters; ++it) {
    float* wc = B.wb[it & 1];
    {
      Timed tm(c, MAPI_K_MAVP);
      HIP_TRY(launch_col_product(o->op, X, D, N, ldx, wc, zpart, z, st, c->stream));
    }
    {
      // the column product sweeps X's rows forward: the row product goes backward from
      // where it ended, and the next column product starts where this one ends
      DenseArgs dl = da;
      dl.reverse = c->alternate ? 1 : 0;
      TimedLaunch tm(c, MAPI_K_MAVP, &dl);
      HIP_TRY(launch_mavp_dense(dl, o->op, z, B.yb[0], B.pp[0], st, NORM_L1, t, c->cu_count, c->stream));
    }
    {
      Timed tm(c, MAPI_K_FINALIZE);
      HIP_TRY(launch_finalize(0, B.yb[0], wc, B.wb[(it & 1) ^ 1], D, st, B.pp[0], P, NORM_L1, B.part, nullptr, 0.0,
                              0.0, c->stream));
    }
    if ((it + 1) % check == 0 && it + 1 < o->max_iters) {
      if ((s = sync_and_state(c, st)) != MAPI_OK) return s;
      if (c->st_host->done) break;
    }
  }
  HIP_TRY(launch_finish(B.wb[0], B.wb[1], w_out, D, st, o->final_l2, c->stream, B.part));
  if ((s = sync_and_state(c, st)) != MAPI_OK) return s;
  fill_info(info, *c->st_host);
  if (info) info->norm *= scale;    // the normaliser of scale * (X (+) z)
  if (c->st_host->status == MAPI_ERR_DEGENERATE)
    return fail(MAPI_ERR_DEGENERATE, "normaliser was zero or not finite after %d iterations", c->st_host->iter);
  return MAPI_OK;
}

mapi_status mapi_quantize(mapi_ctx* c, const float* A, int64_t n_rows, int64_t n_cols, int64_t lda, int32_t dtype,
                          void* out, int64_t ld_out, float* row_scale) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  if (!A || !out) return fail(MAPI_ERR_ARG, "A and out must be device pointers");
  if (n_rows <= 0 || n_cols <= 0 || lda < n_cols || ld_out < n_cols) return fail(MAPI_ERR_ARG, "bad shape");
  HIP_TRY(hipSetDevice(c->device));
  if (dtype == MAPI_BF16) {
    HIP_TRY(launch_quant_bf16(A, n_rows, n_cols, lda, static_cast<uint16_t*>(out), ld_out, c->stream));
  } else if (dtype == MAPI_FP8_E4M3) {
    if (!row_scale) return fail(MAPI_ERR_ARG, "FP8 storage needs row_scale");
    HIP_TRY(launch_quant_fp8(A, n_rows, n_cols, lda, static_cast<uint8_t*>(out), ld_out, row_scale, c->stream));
  } else {
    return fail(MAPI_ERR_ARG, "dtype %d is not a reduced storage format", dtype);
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  return MAPI_OK;
}

// Device memory for the Gram build's float64 partial tiles (none when it runs in one chunk).
static mapi_status gram_ws(mapi_ctx* c, int64_t D, int64_t N, int op, double** out) {
  const size_t need = gram_workspace_bytes(D, N, op);
  *out = nullptr;
  if (need == 0) return MAPI_OK;
  mapi_status s;
  char* base = nullptr;
  if ((s = acquire(c, &c->gws, &c->gws_bytes, need, &base)) != MAPI_OK) return s;
  *out = reinterpret_cast<double*>(base);
  return MAPI_OK;
}

mapi_status mapi_mingram(mapi_ctx* c, const float* X, int64_t D, int64_t N, int64_t ldx, double scale, int32_t op,
                         float* A_out, int64_t lda) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  if (!X || !A_out) return fail(MAPI_ERR_ARG, "X and A_out must be device pointers");
  if (D <= 0 || N <= 0 || ldx < N || lda < D) return fail(MAPI_ERR_ARG, "bad shape");
  if (D > 65536) return fail(MAPI_ERR_UNSUPPORTED, "D > 65536");
  if (!aligned16(X) || ldx % 4 != 0) return fail(MAPI_ERR_ARG, "X base and row pitch must be 16-byte aligned");
  if (op != MAPI_OP_MIN1 && op != MAPI_OP_MIN2 && op != MAPI_OP_DOT) return fail(MAPI_ERR_ARG, "op %d", op);
  HIP_TRY(hipSetDevice(c->device));
  double* gw = nullptr;
  mapi_status s;
  if ((s = gram_ws(c, D, N, op, &gw)) != MAPI_OK) return s;
  {
    Timed tm(c, MAPI_K_GRAM);
    HIP_TRY(launch_gram(X, D, N, ldx, scale, op, A_out, lda, gw, c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  collect_timing(c);
  return MAPI_OK;
}

mapi_status mapi_pca_topk(mapi_ctx* c, const float* X, int64_t D, int64_t N, int64_t ldx, int32_t k, double scale,
                          int32_t method, const float* W0, float* P_out, const mapi_opts* opts, mapi_info* info_k) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  if (!X || !P_out) return fail(MAPI_ERR_ARG, "X and P_out must be device pointers");
  if (D <= 0 || N <= 0 || ldx < N) return fail(MAPI_ERR_ARG, "bad shape");
  if (k < 1 || k > D) return fail(MAPI_ERR_ARG, "k must be in [1, D]");
  if (method != MAPI_METHOD_MAPI && method != MAPI_METHOD_RPI) return fail(MAPI_ERR_ARG, "method %d", method);
  if (!aligned16(X) || ldx % 4 != 0) return fail(MAPI_ERR_ARG, "X base and row pitch must be 16-byte aligned");
  if (D > 32768) return fail(MAPI_ERR_UNSUPPORTED, "D > 32768");
  mapi_status s;
  if ((s = check_opts(opts)) != MAPI_OK) return s;
  HIP_TRY(hipSetDevice(c->device));
  const bool rpi = method == MAPI_METHOD_RPI;
  const int gop = rpi ? MAPI_OP_DOT : opts->op;
  const PcaLayout l = pca_layout(D, k, gram_workspace_bytes(D, N, gop), c->cu_count);
  const int64_t ldA = l.ldA;
  char* base = nullptr;
  if ((s = acquire(c, &c->big, &c->big_bytes, l.total, &base)) != MAPI_OK) return s;
  float* A = reinterpret_cast<float*>(base + l.o_A);
  float* Ai = reinterpret_cast<float*>(base + l.o_Ai);
  double* P = reinterpret_cast<double*>(base + l.o_PQ);
  double* Q = P + (size_t)D * k;
  double* qpart = reinterpret_cast<double*>(base + l.o_qp);
  float* wtmp = reinterpret_cast<float*>(base + l.o_w);
  double* gw = gram_workspace_bytes(D, N, gop) ? reinterpret_cast<double*>(base + l.o_g) : nullptr;
  char* dws = base + l.o_d;
  {
    Timed tm(c, MAPI_K_GRAM);
    HIP_TRY(launch_gram(X, D, N, ldx, scale, gop, A, ldA, gw, c->stream));
  }
  mapi_opts o = *opts;
  o.final_l2 = 0;
  for (int i = 0; i < k; ++i) {
    const float* Acur = A;
    if (i > 0) {
      Timed tm(c, MAPI_K_DEFLATE);
      HIP_TRY(launch_deflate_apply(A, D, ldA, P, Q, i, Ai, ldA, c->stream));
      Acur = Ai;
    }
    mapi_dense desc{Acur, D, D, ldA, MAPI_F32, nullptr};
    mapi_info inf{};
    const float* start = W0 ? W0 + (int64_t)i * D : wtmp;
    if (!W0) HIP_TRY(launch_gen_start((int)D, (uint64_t)i, wtmp, c->stream));   // seeded start, seed i
    s = run_dense(c, &desc, start, wtmp, &o, &inf, rpi, dws);
    if (info_k) info_k[i] = inf;
    if (s != MAPI_OK) return s;
    {
      Timed tm(c, MAPI_K_DEFLATE);
      HIP_TRY(launch_mgs_append(P, D, i, wtmp, P_out + (int64_t)i * D, c->stream));
      HIP_TRY(launch_deflate_q(A, D, ldA, P + (int64_t)i * D, Q + (int64_t)i * D, qpart, c->stream));
    }
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  collect_timing(c);
  return MAPI_OK;
}

mapi_status mapi_image_reconstruct(mapi_ctx* c, const float* V, int64_t P, int32_t N, int64_t ldv, int32_t method,
                                   const float* w0, const mapi_opts* opts, float* R, int64_t ldr, float* W,
                                   mapi_info* info2) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  if (!V || !w0 || !R || !W) return fail(MAPI_ERR_ARG, "V, w0, R and W must be device pointers");
  if (P < 1 || N < 2 || ldv < N || ldr < N) return fail(MAPI_ERR_ARG, "need P >= 1, N >= 2, ldv >= N, ldr >= N");
  if (N > image_max_n()) return fail(MAPI_ERR_UNSUPPORTED, "N > %d images", image_max_n());
  if (P > 32768) return fail(MAPI_ERR_UNSUPPORTED, "P > 32768 pixels");
  if (method != MAPI_METHOD_MAPI && method != MAPI_METHOD_RPI) return fail(MAPI_ERR_ARG, "method %d", method);
  mapi_status s;
  if ((s = check_opts(opts)) != MAPI_OK) return s;
  const bool rpi = method == MAPI_METHOD_RPI;
  if (!rpi && opts->op != MAPI_OP_MIN1 && opts->op != MAPI_OP_MIN2)
    return fail(MAPI_ERR_UNSUPPORTED, "the min-outer deflation is built for the min1 and min2 products");
  if (!aligned16(w0)) return fail(MAPI_ERR_ARG, "w0 must be 16-byte aligned");
  HIP_TRY(hipSetDevice(c->device));
  const int gop = rpi ? MAPI_OP_DOT : opts->op;
  const ImageLayout l = image_layout(P, N, gram_workspace_bytes(P, N, gop), c->cu_count);
  const int64_t ldA = l.ldA, ldc = l.ldc;
  const int G = l.G;
  char* base = nullptr;
  if ((s = acquire(c, &c->big, &c->big_bytes, l.total, &base)) != MAPI_OK) return s;
  float* C = reinterpret_cast<float*>(base + l.o_C);
  float* C2 = reinterpret_cast<float*>(base + l.o_C2);
  float* Vc = reinterpret_cast<float*>(base + l.o_Vc);
  float* m = reinterpret_cast<float*>(base + l.o_m);
  int32_t* perm = reinterpret_cast<int32_t*>(base + l.o_perm);
  double* sums = reinterpret_cast<double*>(base + l.o_sums);
  double* Pm = reinterpret_cast<double*>(base + l.o_P);
  double* Qm = reinterpret_cast<double*>(base + l.o_Q);
  double* qpart = reinterpret_cast<double*>(base + l.o_qp);
  double* gw = gram_workspace_bytes(P, N, gop) ? reinterpret_cast<double*>(base + l.o_g) : nullptr;
  char* dws = base + l.o_d;
  float* w1 = W;
  float* w2 = W + P;
  HIP_TRY(launch_img_center(V, P, N, ldv, Vc, ldc, m, c->stream));
  {
    Timed tm(c, MAPI_K_GRAM);
    HIP_TRY(launch_gram(Vc, P, N, ldc, 1.0 / (double)(N - 1), gop, C, ldA, gw, c->stream));
  }
  // MAPI vectors as Algorithm 1 returns them (l1 units: w (+) w = ||w||_1 = 1 makes
  // w (+) w^T act on w as w w^T does for an l2 unit vector); RPI vectors l2 units
  mapi_opts o = *opts;
  o.final_l2 = rpi ? 1 : 0;
  mapi_dense d1{C, P, P, ldA, MAPI_F32, nullptr};
  mapi_info i1{}, i2{};
  s = run_dense(c, &d1, w0, w1, &o, &i1, rpi, dws);
  if (info2) info2[0] = i1;
  if (s != MAPI_OK) return s;
  {
    Timed tm(c, MAPI_K_DEFLATE);
    if (rpi) {
      HIP_TRY(launch_mgs_append(Pm, P, 0, w1, reinterpret_cast<float*>(base + l.o_pf), c->stream));
      HIP_TRY(launch_deflate_q(C, P, ldA, Pm, Qm, qpart, c->stream));
      HIP_TRY(launch_deflate_apply(C, P, ldA, Pm, Qm, 1, C2, ldA, c->stream));
    } else {
      HIP_TRY(launch_img_minouter_deflate(gop, C, P, ldA, w1, perm, sums, G, C2, c->stream));
    }
  }
  mapi_dense d2{C2, P, P, ldA, MAPI_F32, nullptr};
  s = run_dense(c, &d2, w0, w2, &o, &i2, rpi, dws);
  if (info2) info2[1] = i2;
  if (s != MAPI_OK) return s;
  HIP_TRY(launch_img_reconstruct(gop, W, Vc, P, N, ldc, m, R, ldr, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  collect_timing(c);
  return MAPI_OK;
}

mapi_status mapi_minibatch(mapi_ctx* c, const float* X, int64_t N, int64_t D, int64_t ldx, const int32_t* batch_idx,
                           int32_t s, int32_t T, double beta, int32_t op, int32_t runs, const float* w0, float* w_out,
                           int32_t final_l2, mapi_info* infos) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  if (!X || (!batch_idx && T > 0) || !w0 || !w_out)
    return fail(MAPI_ERR_ARG, "X, batch_idx (when T > 0), w0 and w_out must be device pointers");
  if (N <= 0 || D <= 0 || ldx < D) return fail(MAPI_ERR_ARG, "bad shape");
  if (D > minibatch_max_d()) return fail(MAPI_ERR_UNSUPPORTED, "D > %d", minibatch_max_d());
  if (s < 1 || T < 0 || runs < 1) return fail(MAPI_ERR_ARG, "s >= 1, T >= 0 and runs >= 1 are required");
  if (op != MAPI_OP_MIN1 && op != MAPI_OP_DOT) return fail(MAPI_ERR_ARG, "op must be MAPI_OP_MIN1 or MAPI_OP_DOT");
  if (!(std::fabs(beta) < INFINITY)) return fail(MAPI_ERR_ARG, "beta must be finite");
  HIP_TRY(hipSetDevice(c->device));
  // batch matrices of `range` steps of t are built ahead per launch: the library's choice,
  // or as many as the caller's workspace holds (at least one)
  int range = minibatch_range((int)D, T, runs);
  if (c->user_ws)
    while (range > 1 && minibatch_bytes((int)D, range, runs) > c->user_ws_bytes) range = range / 2;
  Layout L;
  const size_t o_run = L.take(sizeof(MbRun) * (size_t)runs);
  const size_t o_bad = L.take(sizeof(int32_t));
  const size_t o_mb = L.off;
  mapi_status st;
  char* base = nullptr;
  if ((st = acquire(c, &c->ws, &c->ws_bytes, minibatch_bytes((int)D, range, runs), &base)) != MAPI_OK) return st;
  int32_t* bad = reinterpret_cast<int32_t*>(base + o_bad);
  HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int32_t), c->stream));
  {
    Timed tm(c, MAPI_K_MINIBATCH);
    HIP_TRY(launch_minibatch(X, N, (int)D, ldx, batch_idx, s, T, (float)beta, op, runs, w0, w_out, final_l2,
                             reinterpret_cast<MbRun*>(base + o_run), bad, range, base + o_mb, c->stream));
  }
  std::vector<MbRun> host(runs);
  int32_t bad_h = 0;
  HIP_TRY(hipMemcpyAsync(host.data(), base + o_run, sizeof(MbRun) * (size_t)runs, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(&bad_h, bad, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  collect_timing(c);
  if (bad_h) return fail(MAPI_ERR_ARG, "a batch index is outside [0, N)");
  mapi_status worst = MAPI_OK;
  for (int r = 0; r < runs; ++r) {
    if (infos) {
      infos[r].iters = host[r].iters;
      infos[r].converged = 0;
      infos[r].residual = 0.0;
      infos[r].norm = host[r].nu;
      infos[r].status = host[r].status;
    }
    if (host[r].status != MAPI_OK) worst = (mapi_status)host[r].status;
  }
  if (worst != MAPI_OK) return fail(worst, "at least one run stopped on a zero or non-finite normaliser (see infos)");
  return MAPI_OK;
}

mapi_status mapi_pagerank(mapi_ctx* c, const mapi_csr* H, double alpha, int32_t method, const float* w0,
                          float* w_out, const mapi_opts* o, mapi_info* info) {
  return pagerank_run<float>(c, H, alpha, method, w0, w_out, o, info);
}

mapi_status mapi_pagerank_f64(mapi_ctx* c, const mapi_csr* H, double alpha, int32_t method, const double* w0,
                              double* w_out, const mapi_opts* o, mapi_info* info) {
  return pagerank_run<double>(c, H, alpha, method, w0, w_out, o, info);
}

}  // extern "C"
