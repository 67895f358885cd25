// mapi_solve_noalloc: the dense MAPI solve with every device buffer in a static array
// of the library, for callers that cannot allocate device memory.
#include <mutex>

#include "ctx.h"

namespace mapi {

// Largest solve buffer set the array holds (state, partial sums, two iterates and two
// products): n up to about 250000.
constexpr size_t kScratchBytes = size_t(4) << 20;

// One copy of this array exists on every device the library runs on, from the first
// launch there until the process ends.  In host code its name is a host-side stand-in,
// not a device address: host code uses only the address scratch_setup obtains.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char* g_scratch[kMaxDevices] = {};

// This device's address of `scratch` (the device must be current), looked up once per
// device and kept.
mapi_status scratch_setup(int device, char** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return fail(MAPI_ERR_UNSUPPORTED, "device %d beyond %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MAPI_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch[device] = static_cast<char*>(p);
  }
  *out = g_scratch[device];
  return MAPI_OK;
}

}  // namespace mapi

using namespace mapi;

extern "C" mapi_status mapi_solve_noalloc(mapi_ctx* c, const mapi_dense* A, const float* w0, float* w_out,
                                          const mapi_opts* opts, mapi_info* info) {
  if (!c) return fail(MAPI_ERR_ARG, "ctx is NULL");
  mapi_status s;
  if ((s = check_solve_args(A, w0, w_out, opts, false)) != MAPI_OK) return s;
  const size_t need = dense_ws_bytes(A->n_rows, c->cu_count);
  if (need > kScratchBytes)
    return fail(MAPI_ERR_ARG, "mapi_solve_noalloc: n = %lld needs %zu bytes of scratch, the static array holds %zu",
                (long long)A->n_rows, need, kScratchBytes);
  if (!c->scratch) return fail(MAPI_ERR_HIP, "the scratch array's address was not set up by mapi_create");
  HIP_TRY(hipSetDevice(c->device));
  // kernel timing would create events: it is off for this call
  const bool timing = c->timing;
  c->timing = false;
  s = run_dense(c, A, w0, w_out, opts, info, false, c->scratch);
  c->timing = timing;
  return s;
}
