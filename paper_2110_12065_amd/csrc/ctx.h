// Private host-side definitions of libmapi: the context, error reporting,
// device workspace and kernel timing, shared by the C-ABI translation units.
#pragma once

#include <cstdarg>
#include <cstdio>
#include <map>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "common.h"

namespace mapi {
struct BatchState;
struct ServerImpl;
}

namespace mapi {

mapi_status fail(mapi_status s, const char* fmt, ...);

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(MAPI_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

inline int64_t elem_size(int dtype) {
  switch (dtype) {
    case MAPI_F32: return 4;
    case MAPI_BF16: return 2;
    case MAPI_FP8_E4M3: return 1;
    default: return 0;
  }
}

}  // namespace mapi

struct mapi_ctx;
// Frees the batched solver's arena and stream of a context (batch.hip).
void mapi_batch_release(mapi_ctx* c);
// Frees the batched solver's arena only (batch.hip).
mapi_status mapi_batch_free_arena(mapi_ctx* c);

struct mapi_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int cu_count = 256;
  int max_lds = 65536;               // LDS bytes one block may use
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // device workspace given by the caller (mapi_set_workspace): while it is set, every
  // call takes its buffers from it and the context allocates no device memory
  char* user_ws = nullptr;
  size_t user_ws_bytes = 0;
  // this device's copy of the library's static scratch array (mapi_solve_noalloc)
  char* scratch = nullptr;
  // PageRank graphs of at least this many nodes use the column-split product (0: never)
  int64_t csr_split_min_n = int64_t(1) << 20;
  // ... built only after this many plain products of a solve (0: before the first)
  int csr_split_after = 4;
  // dense solves sweep the matrix forward and backward in turn (MAPI_DENSE_ALTERNATE=1);
  // off by default: on MI355X it measured no faster than forward sweeps only
  bool alternate = false;
  // MAPI_DCHECK_SELFTEST=1: dense solves launch one always-failing device check (which
  // only a device-checked build records), to test the reporting path
  bool dcheck_selftest = false;
  mapi::SolveState* st_host = nullptr;     // pinned copy of the device state
  // matrices owned by the PCA driver
  void* big = nullptr;
  size_t big_bytes = 0;
  // intermediate iterate of the MAPI -> RPI hybrid
  void* mid = nullptr;
  size_t mid_bytes = 0;
  // float64 partial tiles of the covariance build
  void* gws = nullptr;
  size_t gws_bytes = 0;
  // timing
  bool timing = false;
  struct Rec { int kind; hipEvent_t a, b; };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  double t_ms[MAPI_K_KINDS] = {};
  int64_t t_n[MAPI_K_KINDS] = {};
  // autotuned launch shapes of the dense product per (dtype, log2 rows, log2 cols)
  std::map<std::tuple<int, int, int>, mapi::DenseTuning> tuned;
  // buckets whose shape the caller set (mapi_tuning_set): their solves always take the
  // multi-kernel path, also where the one-block solve would apply
  std::set<std::tuple<int, int, int>> pinned;
  // persistent batched solver: arena and launch settings
  mapi::BatchState* batch = nullptr;
  hipStream_t side = nullptr;        // stream the batched graph is captured on
  int batch_blocks_per_cu = 2;
  std::map<std::tuple<int, int>, int> batch_rows;   // (dtype, log2 n) -> product tile rows
};

namespace mapi {

inline mapi_status ensure(void** buf, size_t* have, size_t need, mapi_ctx* c) {
  if (*have >= need) return MAPI_OK;
  if (*buf) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipFree(*buf));
    *buf = nullptr;
    *have = 0;
  }
  need = align_up(need, 1 << 20);
  if (hipMalloc(buf, need) != hipSuccess) {
    *buf = nullptr;
    return fail(MAPI_ERR_ALLOC, "hipMalloc of %zu bytes failed", need);
  }
  *have = need;
  return MAPI_OK;
}

// Device memory of one call: `need` bytes of the caller's workspace when one is set
// (MAPI_ERR_ARG if it is smaller), else the context's own buffer *own, grown as needed.
inline mapi_status acquire(mapi_ctx* c, void** own, size_t* have, size_t need, char** out) {
  if (c->user_ws) {
    if (need > c->user_ws_bytes)
      return fail(MAPI_ERR_ARG, "the workspace set by mapi_set_workspace holds %zu bytes; this call needs %zu",
                  c->user_ws_bytes, need);
    *out = c->user_ws;
    return MAPI_OK;
  }
  const mapi_status s = ensure(own, have, need, c);
  if (s != MAPI_OK) return s;
  *out = static_cast<char*>(*own);
  return MAPI_OK;
}

// Bump layout over one allocation, 256-byte aligned pieces.
struct Layout {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  }
};

inline hipEvent_t get_event(mapi_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch with events when timing is enabled.
struct Timed {
  mapi_ctx* c;
  int kind;
  hipEvent_t a = nullptr;
  Timed(mapi_ctx* c_, int k, bool on = true) : c(c_), kind(k) {
    if (on && c->timing) {
      a = get_event(c);
      if (a) (void)hipEventRecord(a, c->stream);
    }
  }
  ~Timed() {
    if (a) {
      hipEvent_t b = get_event(c);
      if (b) {
        (void)hipEventRecord(b, c->stream);
        c->pending.push_back({kind, a, b});
      } else {
        c->pool.push_back(a);
      }
    }
  }
};

// Kernel time of one dense product: the events ride on the launch's own dispatch.
struct TimedLaunch {
  mapi_ctx* c;
  int kind;
  hipEvent_t a = nullptr, b = nullptr;
  // da == nullptr: not timed
  TimedLaunch(mapi_ctx* c_, int k, DenseArgs* da) : c(c_), kind(k) {
    if (da && c->timing) {
      a = get_event(c);
      b = get_event(c);
      if (a && b) {
        da->ev_start = a;
        da->ev_stop = b;
      }
    }
  }
  ~TimedLaunch() {
    if (a && b) {
      c->pending.push_back({kind, a, b});
    } else {
      if (a) c->pool.push_back(a);
      if (b) c->pool.push_back(b);
    }
  }
};

inline void collect_timing(mapi_ctx* c) {
  for (auto& r : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->t_ms[r.kind] += ms;
      c->t_n[r.kind] += 1;
    }
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->pending.clear();
}

// Dense power iteration (api.hip): device bytes of one solve's buffers, the argument
// checks of mapi_solve / rpi_solve, and the solve itself in a region `ws` of
// dense_ws_bytes(n, cu_count) bytes on the context's device (device already current).
size_t dense_ws_bytes(int64_t n, int cu_count);
mapi_status check_solve_args(const mapi_dense* A, const float* w0, const float* w_out, const mapi_opts* o, bool rpi);
mapi_status run_dense(mapi_ctx* c, const mapi_dense* A, const float* w0, float* w_out, const mapi_opts* o,
                      mapi_info* info, bool rpi, char* ws);

// This device's address of the library's static scratch array (noalloc.hip); the
// device must be current.  Called by mapi_create, once per device.
mapi_status scratch_setup(int device, char** out);

inline mapi_status sync_and_state(mapi_ctx* c, const SolveState* st_dev) {
  HIP_TRY(hipMemcpyAsync(c->st_host, st_dev, sizeof(SolveState), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  collect_timing(c);
  if (c->st_host->check != 0)   // only a device-checked build records failures
    return fail(MAPI_ERR_DEVICE_CHECK, "device check failed: file id %u, line %u", c->st_host->check >> 16,
                c->st_host->check & 0xFFFFu);
  return MAPI_OK;
}

}  // namespace mapi
