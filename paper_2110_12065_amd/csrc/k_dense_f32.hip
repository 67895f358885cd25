// Dense product kernels for f32 storage.
#include "dense_kernel.h"

namespace mapi {

hipError_t launch_dense_f32(const DenseArgs& a, int op, const float* w, float* y, double* part, SolveState* st,
                            int norm, const DenseTuning& t, int blocks, hipStream_t s, const FusedPrev* fp) {
  return launch_dt<MAPI_F32>(a, op, w, y, part, st, norm, t, blocks, s, fp);
}

}  // namespace mapi
