// Dense product kernels for fp8 storage.
#include "dense_kernel.h"

namespace mapi {

hipError_t launch_dense_fp8(const DenseArgs& a, int op, const float* w, float* y, double* part, SolveState* st,
                            int norm, const DenseTuning& t, int blocks, hipStream_t s, const FusedPrev* fp) {
  return launch_dt<MAPI_FP8_E4M3>(a, op, w, y, part, st, norm, t, blocks, s, fp);
}

}  // namespace mapi
