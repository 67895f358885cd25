// Arithmetic of the vector products (Sec. 2.1): the min1 / min2 / diamond terms and
// the ordinary product, shared by every product kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mapi.h"

namespace mapi {

// ---------------------------------------------------------------- vector products
// One term of each product, written without multiplication for the min forms:
// with s = signbit(w), x = a ^ s carries sign(a) sign(w), and
//   min1(a, w) = med3(x, -|w|, |w|)   (eq. 3)
//   min2(a, w) = med3(x,  0,   |w|)   (eq. 4)
// The negation and absolute value are free source modifiers of v_med3_f32.
__device__ __forceinline__ float flip_sign(float a, uint32_t s) {
  return __uint_as_float(__float_as_uint(a) ^ s);
}
__device__ __forceinline__ uint32_t sign_bit(float w) { return __float_as_uint(w) & 0x80000000u; }

template <int OP>
__device__ __forceinline__ float op_acc(float acc, float a, float w, uint32_t ws) {
  if constexpr (OP == MAPI_OP_MIN1) {
    const float wa = fabsf(w);
    return acc + __builtin_amdgcn_fmed3f(flip_sign(a, ws), -wa, wa);
  } else if constexpr (OP == MAPI_OP_MIN2) {
    return acc + __builtin_amdgcn_fmed3f(flip_sign(a, ws), 0.0f, fabsf(w));
  } else if constexpr (OP == MAPI_OP_DIAMOND) {
    // eq. (7): sign(a) w + a sign(w); zero when either operand is zero
    const float sa = (a > 0.0f) ? 1.0f : ((a < 0.0f) ? -1.0f : 0.0f);
    const float sw = (w > 0.0f) ? 1.0f : ((w < 0.0f) ? -1.0f : 0.0f);
    return acc + (sa * w + a * sw);
  } else {
    return fmaf(a, w, acc);
  }
}

}  // namespace mapi
