// Serving runtime: continuous batching of MAPI / RPI / PageRank requests on one
// GPU.  A scheduler thread admits requests while an instance slot, device memory
// under the budget and room for the result in a pinned output pool are free; it
// writes the request's descriptor into pinned host memory and one ADMIT item into
// a host-memory inbox that block 0 of the running persistent kernel drains into
// the device queue.  The kernel itself copies the descriptor, and a PageRank
// request's CSR arrays from the caller's pinned host memory, and writes the
// result into the pinned output pool, so admission and completion issue no copy
// command or kernel: nothing of a request waits behind the long-running kernel
// on a shared hardware queue.  A completion thread reads the kernel's completion
// records, copies results to the callers' buffers and frees the request's
// memory.  The kernel is (re)launched from a captured graph whenever admitted
// work exists and no launch is running.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batched.h"
#include "ctx.h"
#include "host_pool.h"

using namespace mapi;

namespace {

using Clock = std::chrono::steady_clock;

struct Ticket {
  mapi_request req{};
  int state = 0;             // 0 queued, 1 admitted, 2 done
  mapi_result res{};
  int slot = -1;
  size_t off = 0, bytes = 0;     // device pool
  size_t out_off = 0;            // pinned output pool (n floats)
  uint32_t tiles = 0;
  // served PageRank request: device-accessible addresses of the caller's pinned arrays
  const int32_t* src_row_ptr = nullptr;
  const int32_t* src_col = nullptr;
  const float* src_val = nullptr;
};

constexpr uint32_t kQueueCap = 1u << 22;
constexpr uint32_t kInboxCap = 1u << 20;

}  // namespace

struct mapi_server {
  mapi_ctx* ctx = nullptr;   // device, tuning tables
  size_t budget = 0;
  int max_slots = 0;
  int blocks = 0;
  double idle_ms = 20.0;
  // device
  char* pool_base = nullptr;
  Pool pool;
  BInst* d_inst = nullptr;
  BQueue* d_q = nullptr;
  BCtl* d_ctl = nullptr;
  unsigned long long* d_item = nullptr;
  // pinned host: descriptors written at admission, results written by the kernel
  BInst* h_stage = nullptr;
  char* out_host = nullptr;
  char* out_dev = nullptr;   // device-accessible address of out_host
  size_t out_bytes = 0;
  Pool out_pool;
  // host-visible (pinned, coherent)
  unsigned long long* inbox = nullptr;
  volatile unsigned long long* inbox_tail = nullptr;
  volatile unsigned long long* inbox_head = nullptr;
  volatile int32_t* quit = nullptr;
  BDone* done = nullptr;
  uint32_t done_cap = 0;
  unsigned long long inbox_pos = 0;
  hipStream_t exec = nullptr, copy = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // bookkeeping
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> queued;
  std::unordered_map<uint64_t, Ticket> tickets;
  std::vector<int> free_slots;
  std::vector<uint64_t> slot_ticket;
  std::vector<int32_t> slot_gen;
  uint64_t next_ticket = 1;
  int64_t live = 0;
  uint64_t live_tiles = 0;
  std::atomic<bool> stop{false};
  std::thread sched, compl_;
  Clock::time_point t0;
  // stats
  int64_t submitted = 0, admitted = 0, completed = 0, rejected = 0, launches = 0;
  std::vector<double> lat_ms;
  double first_submit = -1.0, last_done = 0.0;
  std::string thread_error;
};

namespace {

double ms_since(const mapi_server* s) {
  return std::chrono::duration<double, std::milli>(Clock::now() - s->t0).count();
}

// Device bytes of a request: its instance buffers plus, for PageRank, the CSR copy.
size_t request_bytes(const mapi_request& r, const BInst& I, int64_t mbytes) {
  size_t b = instance_bytes(I, mbytes);
  if (r.prob.kind == MAPI_PROB_CSR)
    b += align_up(sizeof(int32_t) * (size_t)(I.n + 1)) + 2 * align_up(4 * (size_t)r.prob.H.nnz);
  return b;
}

// Device-accessible address of pinned host memory, or NULL when p is not pinned.
const void* pinned_device_address(const void* p) {
  if (!p) return nullptr;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (a.type != hipMemoryTypeHost || !a.devicePointer) return nullptr;
  return a.devicePointer;
}

// Stage one admitted request: lay out its device buffers, write its descriptor to
// the pinned staging slot and queue one ADMIT item.  Host memory writes only.
mapi_status stage(mapi_server* s, Ticket& t, BInst& I, int64_t mbytes) {
  char* base = s->pool_base + t.off;
  char* p = place(&I, base, mbytes);
  I.out = reinterpret_cast<float*>(s->out_dev + t.out_off);
  const mapi_problem& pr = t.req.prob;
  if (pr.kind == MAPI_PROB_CSR) {
    I.row_ptr = reinterpret_cast<int32_t*>(p);
    p += align_up(sizeof(int32_t) * (size_t)(I.n + 1));
    I.col = reinterpret_cast<int32_t*>(p);
    p += align_up(4 * (size_t)pr.H.nnz);
    I.val = reinterpret_cast<float*>(p);
    I.src_row_ptr = t.src_row_ptr;
    I.src_col = t.src_col;
    I.src_val = t.src_val;
  }
  I.prep_err = 0;
  I.arrive = 0;
  I.slot_gen = ++s->slot_gen[t.slot];
  std::memcpy(&s->h_stage[t.slot], &I, sizeof(BInst));
  while (s->inbox_pos + 1 - *s->inbox_head > kInboxCap) {
    if (s->stop) return fail(MAPI_ERR_HIP, "server stopping");
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  std::atomic_thread_fence(std::memory_order_seq_cst);     // descriptor before its item
  s->inbox[s->inbox_pos & (kInboxCap - 1)] = bitem((uint32_t)t.slot, PH_ADMIT, 0);
  std::atomic_thread_fence(std::memory_order_seq_cst);
  s->inbox_pos += 1;
  *s->inbox_tail = s->inbox_pos;
  std::atomic_thread_fence(std::memory_order_seq_cst);
  return MAPI_OK;
}

void finish_ticket(mapi_server* s, Ticket& t, int status) {
  t.res.status = status;
  t.res.t_done_ms = ms_since(s);
  t.state = 2;
}

void scheduler(mapi_server* s) {
  (void)hipSetDevice(s->ctx->device);
  while (!s->stop) {
    bool progressed = false;
    for (;;) {
      uint64_t id;
      Ticket* t;
      BInst I;
      int64_t mbytes = 0;
      {
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->queued.empty()) break;
        id = s->queued.front();
        t = &s->tickets[id];
        const mapi_status d = describe(s->ctx, t->req.prob, &I, &mbytes);
        if (d != MAPI_OK) {
          s->queued.pop_front();
          finish_ticket(s, *t, d);
          ++s->rejected;
          s->cv.notify_all();
          progressed = true;
          continue;
        }
        t->bytes = request_bytes(t->req, I, mbytes);
        t->tiles = max_tiles(I);
        const Admission adm = admit_request(s->pool, s->out_pool, s->budget, t->bytes, sizeof(float) * (size_t)I.n,
                                            !s->free_slots.empty(), s->live_tiles, t->tiles, kQueueCap / 2, &t->off,
                                            &t->out_off);
        if (adm == Admission::kReject) {
          s->queued.pop_front();
          finish_ticket(s, *t, MAPI_ERR_BUDGET);
          ++s->rejected;
          s->cv.notify_all();
          progressed = true;
          continue;
        }
        if (adm == Admission::kWait) break;     // wait for completions to free a slot or memory
        s->queued.pop_front();
        t->slot = s->free_slots.back();
        s->free_slots.pop_back();
        s->slot_ticket[t->slot] = id;
        s->live += 1;
        s->live_tiles += t->tiles;
      }
      const mapi_status st = stage(s, *t, I, mbytes);
      std::unique_lock<std::mutex> lk(s->mu);
      if (st != MAPI_OK) {
        s->pool.release(t->off, t->bytes);
        s->out_pool.release(t->out_off, sizeof(float) * (size_t)I.n);
        s->free_slots.push_back(t->slot);
        s->live -= 1;
        s->live_tiles -= t->tiles;
        finish_ticket(s, *t, st);
        ++s->rejected;
        s->cv.notify_all();
      } else {
        t->state = 1;
        t->res.t_admit_ms = ms_since(s);
        ++s->admitted;
      }
      progressed = true;
    }
    // keep one launch of the persistent kernel running while work is live
    int64_t live;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      live = s->live;
    }
    if (live > 0 && hipStreamQuery(s->exec) == hipSuccess) {
      if (hipGraphLaunch(s->gexec, s->exec) == hipSuccess) {
        std::lock_guard<std::mutex> lk(s->mu);
        ++s->launches;
      }
    }
    if (!progressed) {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait_for(lk, std::chrono::microseconds(200));
    }
  }
}

void completer(mapi_server* s) {
  (void)hipSetDevice(s->ctx->device);
  unsigned long long next = 0;
  for (;;) {
    volatile BDone* d = s->done + (next & (s->done_cap - 1));
    if (d->seq == next + 1) {
      std::atomic_thread_fence(std::memory_order_acquire);
      const int slot = d->slot;
      BDone rec;
      std::memcpy(&rec, const_cast<BDone*>(d), sizeof(BDone));
      Ticket* t;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        t = &s->tickets[s->slot_ticket[slot]];
      }
      const int n = (t->req.prob.kind == MAPI_PROB_CSR) ? (int)t->req.prob.H.n
                    : (t->req.prob.kind == MAPI_PROB_GENERATED ? (int)t->req.prob.gen_n : (int)t->req.prob.A.n_rows);
      // the kernel wrote the result into the pinned output pool (its record follows it)
      if (rec.status == MAPI_OK) std::memcpy(t->req.host_out, s->out_host + t->out_off, sizeof(float) * (size_t)n);
      std::lock_guard<std::mutex> lk(s->mu);
      t->res.iters = rec.iters;
      t->res.converged = rec.converged;
      t->res.residual = rec.residual;
      t->res.norm = rec.norm;
      finish_ticket(s, *t, rec.status);
      s->lat_ms.push_back(t->res.t_done_ms - t->res.t_submit_ms);
      s->last_done = t->res.t_done_ms;
      s->pool.release(t->off, t->bytes);
      s->out_pool.release(t->out_off, sizeof(float) * (size_t)n);
      s->free_slots.push_back(slot);
      s->live -= 1;
      s->live_tiles -= t->tiles;
      ++s->completed;
      ++next;
      s->cv.notify_all();
      continue;
    }
    if (s->stop) {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->live == 0) break;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

void destroy_resources(mapi_server* s) {
  if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  if (s->exec) (void)hipStreamDestroy(s->exec);
  if (s->copy) (void)hipStreamDestroy(s->copy);
  if (s->pool_base) (void)hipFree(s->pool_base);
  if (s->d_inst) (void)hipFree(s->d_inst);
  if (s->inbox) (void)hipHostFree(s->inbox);
  if (s->done) (void)hipHostFree(s->done);
  if (s->h_stage) (void)hipHostFree(s->h_stage);
  if (s->out_host) (void)hipHostFree(s->out_host);
  if (s->ctx) mapi_destroy(s->ctx);
}

void* host_mapped(size_t bytes) {
  void* p = nullptr;
  if (hipHostMalloc(&p, bytes, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) return nullptr;
  std::memset(p, 0, bytes);
  return p;
}

}  // namespace

extern "C" {

mapi_status mapi_serve_create(int device, size_t hbm_budget, const mapi_serve_cfg* cfg, mapi_server** out) {
  if (!out) return fail(MAPI_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (hbm_budget < (1u << 20)) return fail(MAPI_ERR_ARG, "budget below 1 MiB");
  mapi_server* s = new (std::nothrow) mapi_server();
  if (!s) return fail(MAPI_ERR_ALLOC, "server allocation failed");
  mapi_status st = mapi_create(device, nullptr, &s->ctx);
  if (st != MAPI_OK) {
    delete s;
    return st;
  }
  s->budget = hbm_budget;
  s->max_slots = (cfg && cfg->max_slots > 0) ? cfg->max_slots : 2048;
  // Three persistent blocks per compute unit leave a quarter of the register file
  // free, so other work on the device (the caller's own kernels) runs beside the
  // long-lived persistent kernel instead of waiting for it to go idle.
  const int bpc = (cfg && cfg->blocks_per_cu > 0) ? cfg->blocks_per_cu : 2;
  s->blocks = s->ctx->cu_count * bpc;
  s->idle_ms = (cfg && cfg->idle_exit_ms > 0) ? cfg->idle_exit_ms : 20.0;
  if (s->max_slots > (int)kMaxInstances) s->max_slots = (int)kMaxInstances;
  s->done_cap = 1024;
  while (s->done_cap < (uint32_t)(2 * s->max_slots)) s->done_cap <<= 1;
  auto bail = [&](mapi_status code, const char* what) {
    destroy_resources(s);
    delete s;
    return fail(code, "%s", what);
  };
  if (hipMalloc(reinterpret_cast<void**>(&s->pool_base), hbm_budget) != hipSuccess)
    return bail(MAPI_ERR_ALLOC, "could not reserve the memory budget");
  s->pool.reset(hbm_budget);
  Layout L;
  const size_t o_inst = L.take(sizeof(BInst) * s->max_slots);
  const size_t o_q = L.take(sizeof(BQueue));
  const size_t o_ctl = L.take(sizeof(BCtl));
  const size_t o_item = L.take(sizeof(unsigned long long) * kQueueCap);
  char* dev = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&dev), L.off) != hipSuccess) return bail(MAPI_ERR_ALLOC, "device control");
  s->d_inst = reinterpret_cast<BInst*>(dev + o_inst);
  s->d_q = reinterpret_cast<BQueue*>(dev + o_q);
  s->d_ctl = reinterpret_cast<BCtl*>(dev + o_ctl);
  s->d_item = reinterpret_cast<unsigned long long*>(dev + o_item);
  // host-visible control: inbox ring, its two positions, quit flag, completion ring,
  // descriptor staging and the result pool
  s->inbox = static_cast<unsigned long long*>(host_mapped(sizeof(unsigned long long) * (kInboxCap + 32)));
  s->done = static_cast<BDone*>(host_mapped(sizeof(BDone) * s->done_cap));
  s->h_stage = static_cast<BInst*>(host_mapped(sizeof(BInst) * s->max_slots));
  s->out_bytes = std::min<size_t>(hbm_budget, size_t(1) << 30);
  s->out_host = static_cast<char*>(host_mapped(s->out_bytes));
  if (!s->inbox || !s->done || !s->h_stage || !s->out_host) return bail(MAPI_ERR_ALLOC, "pinned host memory");
  s->out_pool.reset(s->out_bytes);
  s->inbox_tail = s->inbox + kInboxCap;
  s->inbox_head = s->inbox + kInboxCap + 8;
  s->quit = reinterpret_cast<volatile int32_t*>(s->inbox + kInboxCap + 16);
  if (hipStreamCreateWithFlags(&s->exec, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) != hipSuccess)
    return bail(MAPI_ERR_HIP, "stream creation");
  BQueue hq{};
  hq.item = s->d_item;
  hq.mask = kQueueCap - 1;
  BCtl hc{};
  hc.mode = 1;
  hc.run_limit = 5 * realtime_hz();
  hc.idle_limit = (int64_t)(s->idle_ms * 1e-3 * (double)realtime_hz());
  void* dp = nullptr;
  if (hipHostGetDevicePointer(&dp, s->inbox, 0) != hipSuccess) return bail(MAPI_ERR_HIP, "inbox mapping");
  hc.inbox = static_cast<const unsigned long long*>(dp);
  hc.inbox_tail = static_cast<const volatile unsigned long long*>(dp) + kInboxCap;
  hc.inbox_head_host = static_cast<volatile unsigned long long*>(dp) + kInboxCap + 8;
  hc.quit = reinterpret_cast<const volatile int32_t*>(static_cast<unsigned long long*>(dp) + kInboxCap + 16);
  hc.inbox_mask = kInboxCap - 1;
  if (hipHostGetDevicePointer(&dp, s->done, 0) != hipSuccess) return bail(MAPI_ERR_HIP, "completion mapping");
  hc.done = static_cast<BDone*>(dp);
  if (hipHostGetDevicePointer(&dp, s->h_stage, 0) != hipSuccess) return bail(MAPI_ERR_HIP, "staging mapping");
  hc.inst_stage = static_cast<const BInst*>(dp);
  if (hipHostGetDevicePointer(&dp, s->out_host, 0) != hipSuccess) return bail(MAPI_ERR_HIP, "output mapping");
  s->out_dev = static_cast<char*>(dp);
  hc.done_mask = s->done_cap - 1;
  if (hipMemsetAsync(s->d_item, 0, sizeof(unsigned long long) * kQueueCap, s->copy) != hipSuccess ||
      hipMemcpyAsync(s->d_q, &hq, sizeof(hq), hipMemcpyHostToDevice, s->copy) != hipSuccess ||
      hipMemcpyAsync(s->d_ctl, &hc, sizeof(hc), hipMemcpyHostToDevice, s->copy) != hipSuccess ||
      hipStreamSynchronize(s->copy) != hipSuccess)
    return bail(MAPI_ERR_HIP, "control upload");
  if (hipStreamBeginCapture(s->exec, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return bail(MAPI_ERR_HIP, "graph capture");
  const hipError_t le = launch_persistent(s->d_q, s->d_inst, s->d_ctl, s->blocks, s->exec);
  const hipError_t ce = hipStreamEndCapture(s->exec, &s->graph);
  if (le != hipSuccess || ce != hipSuccess || hipGraphInstantiate(&s->gexec, s->graph, nullptr, nullptr, 0) != hipSuccess)
    return bail(MAPI_ERR_HIP, "graph instantiation");
  s->slot_ticket.assign(s->max_slots, 0);
  s->slot_gen.assign(s->max_slots, 0);
  for (int i = s->max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
  s->t0 = Clock::now();
  s->sched = std::thread(scheduler, s);
  s->compl_ = std::thread(completer, s);
  *out = s;
  return MAPI_OK;
}

mapi_status mapi_serve_submit(mapi_server* s, const mapi_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return fail(MAPI_ERR_ARG, "NULL argument");
  if (!req->host_out) return fail(MAPI_ERR_ARG, "host_out is NULL");
  BInst I;
  int64_t mb = 0;
  mapi_status st = describe(s->ctx, req->prob, &I, &mb);
  if (st != MAPI_OK) return st;
  if (request_bytes(*req, I, mb) > s->budget) return fail(MAPI_ERR_BUDGET, "request needs more than the budget");
  if (sizeof(float) * (size_t)I.n > s->out_bytes) return fail(MAPI_ERR_BUDGET, "result larger than the output pool");
  const void* src[3] = {nullptr, nullptr, nullptr};
  if (req->prob.kind == MAPI_PROB_CSR) {
    const mapi_csr& H = req->prob.H;
    src[0] = pinned_device_address(H.row_ptr);
    src[1] = H.nnz ? pinned_device_address(H.col) : nullptr;
    src[2] = H.nnz ? pinned_device_address(H.val) : nullptr;
    if (!src[0] || (H.nnz && (!src[1] || !src[2])))
      return fail(MAPI_ERR_ARG, "CSR arrays of a served request must be in pinned host memory (hipHostMalloc)");
  }
  std::lock_guard<std::mutex> lk(s->mu);
  const uint64_t id = s->next_ticket++;
  Ticket& t = s->tickets[id];
  t.req = *req;
  t.src_row_ptr = static_cast<const int32_t*>(src[0]);
  t.src_col = static_cast<const int32_t*>(src[1]);
  t.src_val = static_cast<const float*>(src[2]);
  t.res.t_submit_ms = ms_since(s);
  if (s->first_submit < 0) s->first_submit = t.res.t_submit_ms;
  s->queued.push_back(id);
  ++s->submitted;
  *ticket = id;
  s->cv.notify_all();
  return MAPI_OK;
}

mapi_status mapi_serve_poll(mapi_server* s, uint64_t ticket, mapi_result* res) {
  if (!s) return fail(MAPI_ERR_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(MAPI_ERR_ARG, "unknown ticket");
  if (it->second.state != 2) return MAPI_ERR_PENDING;
  if (res) *res = it->second.res;
  return MAPI_OK;
}

mapi_status mapi_serve_wait(mapi_server* s, uint64_t ticket, int64_t timeout_us, mapi_result* res) {
  if (!s) return fail(MAPI_ERR_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(MAPI_ERR_ARG, "unknown ticket");
  const auto until = Clock::now() + std::chrono::microseconds(timeout_us < 0 ? 0 : timeout_us);
  while (it->second.state != 2) {
    if (timeout_us < 0) {
      s->cv.wait_for(lk, std::chrono::milliseconds(5));
    } else {
      if (Clock::now() >= until) return MAPI_ERR_TIMEOUT;
      s->cv.wait_until(lk, until);
    }
  }
  if (res) *res = it->second.res;
  return MAPI_OK;
}

mapi_status mapi_serve_stats(mapi_server* s, mapi_serve_summary* o) {
  if (!s || !o) return fail(MAPI_ERR_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *o = mapi_serve_summary{};
  o->submitted = s->submitted;
  o->admitted = s->admitted;
  o->completed = s->completed;
  o->rejected = s->rejected;
  o->budget_bytes = s->budget;
  o->peak_bytes = s->pool.peak();
  o->kernel_launches = s->launches;
  if (s->completed > 0 && s->last_done > s->first_submit)
    o->solves_per_s = (double)s->completed / ((s->last_done - s->first_submit) * 1e-3);
  if (!s->lat_ms.empty()) {
    std::vector<double> v = s->lat_ms;
    std::sort(v.begin(), v.end());
    auto q = [&](double f) { return v[std::min(v.size() - 1, (size_t)(f * (double)(v.size() - 1) + 0.5))]; };
    o->p50_ms = q(0.50);
    o->p99_ms = q(0.99);
  }
  return MAPI_OK;
}

void mapi_serve_destroy(mapi_server* s) {
  if (!s) return;
  // let admitted and queued work finish (at most a minute), then stop
  const auto give_up = Clock::now() + std::chrono::seconds(60);
  while (Clock::now() < give_up) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->queued.empty() && s->live == 0) break;
    }
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->live = 0;            // the completion thread must not wait for abandoned work
  }
  *s->quit = 1;
  s->stop = true;
  s->cv.notify_all();
  if (s->sched.joinable()) s->sched.join();
  if (s->compl_.joinable()) s->compl_.join();
  (void)hipStreamSynchronize(s->exec);
  destroy_resources(s);
  delete s;
}

}  // extern "C"
