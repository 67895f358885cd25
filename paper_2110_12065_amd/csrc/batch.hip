// Host runtime of the persistent batched solver: instance layout, the device
// arena, the captured launch graph and the row-split autotuner.
#include <algorithm>
#include <cstddef>
#include <chrono>
#include <cmath>
#include <vector>

#include "batched.h"
#include "ctx.h"

using namespace mapi;

namespace mapi {

struct BatchState {
  void* arena = nullptr;
  size_t bytes = 0;
};

int batch_default_rows(int kind, int dtype, int64_t n) {
  if (kind == BK_CSR) return (int)std::max<int64_t>(1024, (n + kMaxTiles - 1) / kMaxTiles);
  const int64_t es = elem_size(dtype);
  // About 1 MiB of matrix per tile: every item costs a few device-wide fences and a
  // claim on one counter, which the whole chip serialises, so items must be large.
  int64_t r = (1024 * 1024) / std::max<int64_t>(1, n * es);
  r = std::max<int64_t>(4, std::min<int64_t>(r, kMaxTileRows));
  return (int)((r + 3) / 4 * 4);
}

static int log2ceil(int64_t x) {
  int k = 0;
  while ((int64_t(1) << k) < x) ++k;
  return k;
}

int batch_rows_for(mapi_ctx* c, int kind, int dtype, int64_t n) {
  if (kind != BK_CSR) {
    auto it = c->batch_rows.find(std::make_tuple(dtype, log2ceil(n)));
    if (it != c->batch_rows.end()) return it->second;
  }
  return batch_default_rows(kind, dtype, n);
}

// Fill the static part of an instance from a problem; device buffers are set later.
mapi_status describe(mapi_ctx* c, const mapi_problem& p, BInst* I, int64_t* matrix_bytes) {
  *I = BInst{};
  I->method = p.method;
  I->op = p.opts.op;
  I->max_iters = p.opts.max_iters;
  I->stall_iters = p.opts.stall_iters;
  I->tol = p.opts.tol;
  I->w0 = p.w0;
  I->out = p.w_out;
  I->seed = p.seed;
  *matrix_bytes = 0;
  if (p.method != MAPI_METHOD_MAPI && p.method != MAPI_METHOD_RPI) return fail(MAPI_ERR_ARG, "method %d", p.method);
  if (p.opts.max_iters < 0 || !(p.opts.tol >= 0.0) || p.opts.stall_iters < 0) return fail(MAPI_ERR_ARG, "bad opts");
  if (p.opts.final_l2) return fail(MAPI_ERR_UNSUPPORTED, "final_l2 is not available in batched solves");
  if (p.method == MAPI_METHOD_MAPI && p.opts.op != MAPI_OP_MIN1 && p.opts.op != MAPI_OP_MIN2)
    return fail(MAPI_ERR_UNSUPPORTED, "batched MAPI supports the min1 and min2 products");
  int64_t n = 0;
  if (p.kind == MAPI_PROB_DENSE) {
    const mapi_dense& A = p.A;
    if (!A.data || A.n_rows <= 0 || A.n_rows != A.n_cols || A.ld < A.n_cols || !elem_size(A.dtype))
      return fail(MAPI_ERR_ARG, "dense problem needs a square matrix");
    if (!aligned16(A.data) || (A.ld * elem_size(A.dtype)) % 16) return fail(MAPI_ERR_ARG, "matrix must be 16-byte aligned");
    if (A.dtype == MAPI_FP8_E4M3 && !A.row_scale) return fail(MAPI_ERR_ARG, "FP8 storage needs row_scale");
    n = A.n_rows;
    I->kind = BK_DENSE;
    I->dtype = A.dtype;
    I->A = A.data;
    I->ld = A.ld;
    I->row_scale = A.row_scale;
  } else if (p.kind == MAPI_PROB_CSR) {
    if (!p.H.row_ptr || p.H.n <= 0 || p.H.nnz < 0 || (p.H.nnz > 0 && (!p.H.col || !p.H.val)))
      return fail(MAPI_ERR_ARG, "bad CSR problem");
    if (!(p.alpha > 0.0 && p.alpha < 1.0)) return fail(MAPI_ERR_ARG, "alpha must be in (0, 1)");
    n = p.H.n;
    I->kind = BK_CSR;
    I->dtype = MAPI_F32;
    I->row_ptr = p.H.row_ptr;
    I->col = p.H.col;
    I->val = p.H.val;
    I->alpha = (float)p.alpha;
    I->inv_n = 1.0 / (double)n;
    I->c = (float)((1.0 - p.alpha) * I->inv_n);
    I->nnz = p.H.nnz;
    I->etiles = (int32_t)((p.H.nnz + kEdgeTile - 1) / kEdgeTile);
  } else if (p.kind == MAPI_PROB_GENERATED) {
    if (p.gen_n <= 0 || p.gen_n > 16384) return fail(MAPI_ERR_ARG, "generated size must be in [1, 16384]");
    if (p.gen_dtype != MAPI_F32 && p.gen_dtype != MAPI_BF16) return fail(MAPI_ERR_ARG, "generated storage F32 or BF16");
    n = p.gen_n;
    I->kind = BK_GEN;
    I->dtype = p.gen_dtype;
    I->ld = (n + 7) / 8 * 8;
    *matrix_bytes = I->ld * n * elem_size(p.gen_dtype);
    const GenConsts g = gen_consts(n);
    I->gen_scale = g.scale;
    I->gen_spike = g.spike;
    I->gen_w0 = g.w0;
  } else {
    return fail(MAPI_ERR_ARG, "unknown problem kind %d", p.kind);
  }
  if (n > INT32_MAX / 2) return fail(MAPI_ERR_ARG, "problem too large");
  I->n = (int)n;
  I->rows_per_tile = batch_rows_for(c, I->kind, I->dtype, n);
  I->ntiles = (int)((n + I->rows_per_tile - 1) / I->rows_per_tile);
  I->vtiles = (int)((n + kVecTile - 1) / kVecTile);
  I->gtiles = I->kind == BK_GEN ? (int)((n + kGenRows - 1) / kGenRows) : 0;
  if ((uint32_t)std::max(std::max(I->ntiles, I->vtiles), std::max(I->gtiles, I->etiles)) > kMaxTiles)
    return fail(MAPI_ERR_UNSUPPORTED, "problem needs more than %u tiles per phase", kMaxTiles);
  I->solo = I->ntiles == 1 ? 1 : 0;
  SolveState& st = I->st;
  st = SolveState{};
  st.best_r = INFINITY;
  st.tol = p.opts.tol;
  st.max_iters = p.opts.max_iters;
  st.stall_iters = p.opts.stall_iters;
  return MAPI_OK;
}

// Device bytes an instance needs besides its inputs: iterates, product, partials,
// dangling flags, generated matrix.
size_t instance_bytes(const BInst& I, int64_t matrix_bytes) {
  size_t b = 3 * align_up(sizeof(float) * (size_t)I.n) + align_up(sizeof(double) * (I.ntiles + 3 * I.vtiles));
  if (I.kind == BK_CSR) b += align_up((size_t)I.n);
  return b + align_up((size_t)matrix_bytes);
}

// Carve an instance's buffers out of `base` (layout of instance_bytes).
char* place(BInst* I, char* base, int64_t matrix_bytes) {
  I->wb0 = reinterpret_cast<float*>(base);
  base += align_up(sizeof(float) * (size_t)I->n);
  I->wb1 = reinterpret_cast<float*>(base);
  base += align_up(sizeof(float) * (size_t)I->n);
  I->y = reinterpret_cast<float*>(base);
  base += align_up(sizeof(float) * (size_t)I->n);
  I->part = reinterpret_cast<double*>(base);
  base += align_up(sizeof(double) * (I->ntiles + 3 * I->vtiles));
  if (I->kind == BK_CSR) {
    I->dangling = reinterpret_cast<uint8_t*>(base);
    base += align_up((size_t)I->n);
  }
  if (matrix_bytes) {
    I->A = base;
    base += align_up((size_t)matrix_bytes);
  }
  return base;
}

uint32_t first_phase_tiles(const BInst& I, int* phase) {
  if (I.kind == BK_GEN) {
    *phase = PH_GEN;
    return (uint32_t)I.gtiles;
  }
  *phase = PH_INIT;
  return (uint32_t)I.vtiles;
}

uint32_t max_tiles(const BInst& I) {
  return (uint32_t)std::max(std::max(I.ntiles, I.vtiles), std::max(std::max(I.gtiles, I.etiles), 1));
}

uint32_t pow2_at_least(uint64_t x) {
  uint64_t c = 1024;
  while (c < x) c <<= 1;
  return (uint32_t)c;
}

int64_t realtime_hz() { return 100000000; }   // s_memrealtime runs at 100 MHz on CDNA

}  // namespace mapi

mapi_status mapi_batch_free_arena(mapi_ctx* c) {
  if (c->batch && c->batch->arena) {
    HIP_TRY(hipFree(c->batch->arena));
    c->batch->arena = nullptr;
    c->batch->bytes = 0;
  }
  return MAPI_OK;
}

void mapi_batch_release(mapi_ctx* c) {
  if (c->batch) {
    if (c->batch->arena) (void)hipFree(c->batch->arena);
    delete c->batch;
    c->batch = nullptr;
  }
  if (c->side) {
    (void)hipStreamDestroy(c->side);
    c->side = nullptr;
  }
}

extern "C" {

mapi_status mapi_batched_config(mapi_ctx* c, int32_t blocks_per_cu) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  if (blocks_per_cu < 1 || blocks_per_cu > 8) return fail(MAPI_ERR_ARG, "blocks_per_cu must be in 1..8");
  c->batch_blocks_per_cu = blocks_per_cu;
  return MAPI_OK;
}

mapi_status mapi_batched_rows_set(mapi_ctx* c, int32_t dtype, int64_t n, int32_t rows) {
  if (!c || n <= 0 || !elem_size(dtype) || rows < 1) return fail(MAPI_ERR_ARG, "bad arguments");
  c->batch_rows[std::make_tuple((int)dtype, log2ceil(n))] = rows;
  return MAPI_OK;
}

mapi_status mapi_batched_rows_get(mapi_ctx* c, int32_t dtype, int64_t n, int32_t* rows) {
  if (!c || n <= 0 || !elem_size(dtype) || !rows) return fail(MAPI_ERR_ARG, "bad arguments");
  *rows = batch_rows_for(c, BK_DENSE, dtype, n);
  return MAPI_OK;
}

mapi_status mapi_generate_dense(mapi_ctx* c, int64_t n, uint64_t seed, float* A, int64_t ld, float* w0) {
  if (!c || !A || n <= 0 || n > 16384 || ld < n) return fail(MAPI_ERR_ARG, "bad arguments");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(launch_gen_dense((int)n, seed, A, ld, w0, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return MAPI_OK;
}

// Arena of one batched solve: instances, queue, control block, queue items, error
// flags, then every instance's buffers.  Fills H and mbytes from the problems.
struct ArenaLayout {
  uint32_t cap;
  size_t o_inst, o_q, o_ctl, o_item, o_err, o_bufs, total;
};
static mapi_status batch_layout(mapi_ctx* c, int32_t count, const mapi_problem* probs, std::vector<BInst>& H,
                                std::vector<int64_t>& mbytes, ArenaLayout* a) {
  if (count < 1 || !probs) return fail(MAPI_ERR_ARG, "bad arguments");
  if ((uint32_t)count > kMaxInstances) return fail(MAPI_ERR_ARG, "too many instances");
  H.assign(count, BInst{});
  mbytes.assign(count, 0);
  uint64_t items = 0, first_items = 0;
  size_t inst_total = 0;
  mapi_status s;
  for (int i = 0; i < count; ++i) {
    if ((s = describe(c, probs[i], &H[i], &mbytes[i])) != MAPI_OK) return fail(s, "problem %d: %s", i, mapi_last_error());
    int ph;
    first_items += first_phase_tiles(H[i], &ph);
    items += max_tiles(H[i]);
    inst_total += instance_bytes(H[i], mbytes[i]);
  }
  a->cap = pow2_at_least(items + first_items + 64);
  Layout L;
  a->o_inst = L.take(sizeof(BInst) * count);
  a->o_q = L.take(sizeof(BQueue));
  a->o_ctl = L.take(sizeof(BCtl));
  a->o_item = L.take(sizeof(unsigned long long) * a->cap);
  a->o_err = L.take(sizeof(int32_t) * count);
  a->o_bufs = L.take(inst_total);
  a->total = L.off;
  return MAPI_OK;
}

mapi_status mapi_solve_batched_workspace_size(mapi_ctx* c, int32_t count, const mapi_problem* probs, size_t* bytes) {
  if (!c || !bytes) return fail(MAPI_ERR_ARG, "ctx and bytes are required");
  *bytes = 0;
  if (count == 0) return MAPI_OK;
  std::vector<BInst> H;
  std::vector<int64_t> mbytes;
  ArenaLayout a;
  const mapi_status s = batch_layout(c, count, probs, H, mbytes, &a);
  if (s == MAPI_OK) *bytes = a.total;
  return s;
}

mapi_status mapi_solve_batched(mapi_ctx* c, int32_t count, const mapi_problem* probs, mapi_info* infos) {
  if (!c || count < 0 || (count > 0 && !probs)) return fail(MAPI_ERR_ARG, "bad arguments");
  if (count == 0) return MAPI_OK;
  HIP_TRY(hipSetDevice(c->device));
  mapi_status s;
  std::vector<BInst> H;
  std::vector<int64_t> mbytes;
  ArenaLayout a;
  if ((s = batch_layout(c, count, probs, H, mbytes, &a)) != MAPI_OK) return s;
  for (int i = 0; i < count; ++i)
    if (!probs[i].w_out) return fail(MAPI_ERR_ARG, "problem %d: w_out is NULL", i);
  const uint32_t cap = a.cap;
  const size_t o_inst = a.o_inst, o_q = a.o_q, o_ctl = a.o_ctl, o_item = a.o_item, o_err = a.o_err, o_bufs = a.o_bufs;
  if (!c->batch) c->batch = new BatchState();
  char* base = nullptr;
  if ((s = acquire(c, &c->batch->arena, &c->batch->bytes, a.total, &base)) != MAPI_OK) return s;
  BInst* d_inst = reinterpret_cast<BInst*>(base + o_inst);
  BQueue* d_q = reinterpret_cast<BQueue*>(base + o_q);
  BCtl* d_ctl = reinterpret_cast<BCtl*>(base + o_ctl);
  unsigned long long* d_item = reinterpret_cast<unsigned long long*>(base + o_item);
  int32_t* d_err = reinterpret_cast<int32_t*>(base + o_err);
  char* buf = base + o_bufs;
  for (int i = 0; i < count; ++i) buf = place(&H[i], buf, mbytes[i]);

  if (!c->side) HIP_TRY(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
  hipStream_t ss = c->side;
  // inputs come from the caller's stream
  hipEvent_t ready = get_event(c);
  if (!ready) return fail(MAPI_ERR_HIP, "event creation failed");
  HIP_TRY(hipEventRecord(ready, c->stream));
  HIP_TRY(hipStreamWaitEvent(ss, ready, 0));
  c->pool.push_back(ready);

  // PageRank inputs: validate and mark dangling nodes
  HIP_TRY(hipMemsetAsync(d_err, 0, sizeof(int32_t) * count, ss));
  for (int i = 0; i < count; ++i)
    if (H[i].kind == BK_CSR)
      HIP_TRY(launch_csr_prep(H[i].row_ptr, H[i].col, H[i].n, probs[i].H.nnz, const_cast<uint8_t*>(H[i].dangling),
                              d_err + i, ss));
  std::vector<int32_t> errs(count);
  HIP_TRY(hipMemcpyAsync(errs.data(), d_err, sizeof(int32_t) * count, hipMemcpyDeviceToHost, ss));

  // queue: the first phase of every instance, in instance order
  std::vector<unsigned long long> h_item(cap, 0ull);
  unsigned long long pos = 0;
  for (int i = 0; i < count; ++i) {
    int ph;
    const uint32_t t = first_phase_tiles(H[i], &ph);
    for (uint32_t k = 0; k < t; ++k, ++pos) h_item[pos] = bslot(pos, bitem((uint32_t)i, ph, k));
  }
  BQueue hq{};
  hq.head = 0;
  hq.tail = pos;
  hq.item = d_item;
  hq.mask = cap - 1;
  hq.live = (uint32_t)count;
  BCtl hc{};
  hc.mode = 0;
  hc.run_limit = 60 * realtime_hz();
  hc.idle_limit = realtime_hz() / 200;   // 5 ms without work
  HIP_TRY(hipMemcpyAsync(d_inst, H.data(), sizeof(BInst) * count, hipMemcpyHostToDevice, ss));
  HIP_TRY(hipMemcpyAsync(d_item, h_item.data(), sizeof(unsigned long long) * cap, hipMemcpyHostToDevice, ss));
  HIP_TRY(hipMemcpyAsync(d_q, &hq, sizeof(BQueue), hipMemcpyHostToDevice, ss));
  HIP_TRY(hipMemcpyAsync(d_ctl, &hc, sizeof(BCtl), hipMemcpyHostToDevice, ss));
  HIP_TRY(hipStreamSynchronize(ss));
  for (int i = 0; i < count; ++i)
    if (errs[i]) return fail(MAPI_ERR_ARG, "problem %d: invalid CSR arrays (code %d)", i, errs[i]);

  // one captured launch of the persistent kernel
  const int blocks = c->cu_count * c->batch_blocks_per_cu;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  HIP_TRY(hipStreamBeginCapture(ss, hipStreamCaptureModeThreadLocal));
  const hipError_t le = launch_persistent(d_q, d_inst, d_ctl, blocks, ss);
  const hipError_t ce = hipStreamEndCapture(ss, &graph);
  if (le != hipSuccess || ce != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(MAPI_ERR_HIP, "graph capture failed: %s", hipGetErrorString(le != hipSuccess ? le : ce));
  }
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(MAPI_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
  }
  BQueue qs{};
  int launches = 0;
  for (;;) {
    hipEvent_t a = nullptr, b = nullptr;
    if (c->timing) {
      a = get_event(c);
      b = get_event(c);
      if (a) (void)hipEventRecord(a, ss);
    }
    e = hipGraphLaunch(exec, ss);
    if (e == hipSuccess && b) e = hipEventRecord(b, ss);
    if (e == hipSuccess) e = hipMemcpyAsync(&qs, d_q, sizeof(BQueue), hipMemcpyDeviceToHost, ss);
    if (e == hipSuccess) e = hipStreamSynchronize(ss);
    if (a && b) c->pending.push_back({MAPI_K_BATCHED, a, b});
    ++launches;
    if (e != hipSuccess || qs.live == 0 || launches >= 32) break;
    // blocks stopped at the run limit with work queued: launch again
    const uint32_t zero = 0;
    e = hipMemcpyAsync(reinterpret_cast<char*>(d_q) + offsetof(BQueue, error), &zero, sizeof(zero),
                       hipMemcpyHostToDevice, ss);
    if (e != hipSuccess) break;
  }
  (void)hipGraphExecDestroy(exec);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(MAPI_ERR_HIP, "persistent kernel: %s", hipGetErrorString(e));
  collect_timing(c);
  if (qs.live != 0) return fail(MAPI_ERR_HIP, "%u instances unfinished after %d launches", qs.live, launches);
  HIP_TRY(hipMemcpy(H.data(), d_inst, sizeof(BInst) * count, hipMemcpyDeviceToHost));
  mapi_status worst = MAPI_OK;
  for (int i = 0; i < count; ++i) {
    if (infos) {
      infos[i].iters = H[i].st.iter;
      infos[i].converged = H[i].st.converged;
      infos[i].residual = H[i].st.r;
      infos[i].norm = H[i].st.nu;
      infos[i].status = H[i].st.status;
    }
    if (H[i].st.status != MAPI_OK) worst = (mapi_status)H[i].st.status;
    if (H[i].st.check != 0)   // only a device-checked build records failures
      return fail(MAPI_ERR_DEVICE_CHECK, "device check failed in instance %d: file id %u, line %u", i,
                  H[i].st.check >> 16, H[i].st.check & 0xFFFFu);
  }
  if (worst != MAPI_OK) return fail(worst, "at least one instance failed (see infos)");
  return MAPI_OK;
}

mapi_status mapi_autotune_batched(mapi_ctx* c, int32_t dtype, int64_t n, int32_t count, int32_t iters,
                                  int32_t* best_rows, double* best_ms) {
  if (!c || n <= 0 || n > 16384 || count < 1 || iters < 1) return fail(MAPI_ERR_ARG, "bad arguments");
  if (dtype != MAPI_F32 && dtype != MAPI_BF16) return fail(MAPI_ERR_ARG, "dtype F32 or BF16");
  HIP_TRY(hipSetDevice(c->device));
  // the candidates' results: the tail of the caller's workspace (the solves get the
  // rest), else a temporary allocation
  float* out = nullptr;
  const size_t out_bytes = align_up(sizeof(float) * (size_t)n * count);
  char* const user_ws = c->user_ws;
  const size_t user_bytes = c->user_ws_bytes;
  if (user_ws) {
    if (user_bytes < out_bytes) return fail(MAPI_ERR_ARG, "the workspace set by mapi_set_workspace is too small");
    c->user_ws_bytes = (user_bytes - out_bytes) / 256 * 256;
    out = reinterpret_cast<float*>(user_ws + c->user_ws_bytes);
  } else {
    HIP_TRY(hipMalloc(&out, sizeof(float) * (size_t)n * count));
  }
  std::vector<mapi_problem> P(count);
  for (int i = 0; i < count; ++i) {
    mapi_problem p{};
    p.kind = MAPI_PROB_GENERATED;
    p.method = MAPI_METHOD_MAPI;
    p.gen_n = n;
    p.gen_dtype = dtype;
    p.seed = 1000003ull * (i + 1);
    p.w_out = out + (size_t)n * i;
    p.opts.max_iters = iters;
    p.opts.op = MAPI_OP_MIN1;
    P[i] = p;
  }
  const auto key = std::make_tuple((int)dtype, log2ceil(n));
  const auto saved = c->batch_rows.find(key) != c->batch_rows.end() ? c->batch_rows[key] : -1;
  int best = batch_default_rows(BK_DENSE, dtype, n);
  double bms = 1e30;
  mapi_status s = MAPI_OK;
  for (int rows : {4, 8, 16, 32, 64, 128, 256, 512, 1024}) {
    if (rows > n && rows != 4) continue;
    c->batch_rows[key] = rows;
    const auto t0 = std::chrono::steady_clock::now();
    s = mapi_solve_batched(c, count, P.data(), nullptr);
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (s != MAPI_OK) break;
    if (ms < bms) {
      bms = ms;
      best = rows;
    }
  }
  if (user_ws) c->user_ws_bytes = user_bytes;
  else (void)hipFree(out);
  if (s != MAPI_OK) {
    if (saved > 0) c->batch_rows[key] = saved;
    else c->batch_rows.erase(key);
    return s;
  }
  c->batch_rows[key] = best;
  if (best_rows) *best_rows = best;
  if (best_ms) *best_ms = bms;
  return MAPI_OK;
}

}  // extern "C"
