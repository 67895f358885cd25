// Whole power iteration of a small dense float32 system in one block (Algorithm 1
// for MAPI, eq. 1 for RPI, n <= 256).  At this size a solve is bound by launch and
// synchronisation latency, not by memory: one launch per iteration pair costs more
// than the iteration's arithmetic.  Here the matrix is read once into registers and
// every iteration runs inside the kernel: the product, the float64 normaliser, the
// residual ||w_t - w_{t-1}||_1 and the stop rule, with the same arithmetic per
// element as the multi-kernel path (w = fl32(y * (1 / nu)), float64 sums of |y| or
// y^2 and of the residual); only the order of the float32 row sums and the float64
// sums differs.
#include "common.h"

namespace mapi {

constexpr int kSmallN = 256;                    // largest n
constexpr int kSmallThreads = 1024;
constexpr int kSmallRows = kSmallN / (kSmallThreads / kWave);   // rows per wave (16)

// One halving step at lane bit 5 (B = 32) or 4 (B = 16) by a lane swap between two
// registers: v_permlane32_swap exchanges lanes 32..63 of `lo` with lanes 0..31 of `hi`,
// v_permlane16_swap the odd 16-lane rows of `lo` with the even rows of `hi`.  Afterwards
// a lane whose bit B is clear holds its own `lo` and its partner's `lo`, a lane whose bit
// is set its partner's `hi` and its own `hi`: the sum is the halved partial.
template <int B>
__device__ __forceinline__ float swap_halve(float lo, float hi) {
  const auto r = B == 32 ? __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false)
                         : __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Reduce-scatter of 16 row partials over the wave.  Each halving step pairs every lane
// with a partner that differs in the step's lane bit and agrees in the bits halved
// before: bits 5 and 4 by lane swaps, bit 3 by row_mirror, bit 2 by row_half_mirror.  A lane keeps the half of its partials that
// its bit selects and adds the partner's partials of that half.  The partials of rows
// j and j + 8 are formed together and halved at once, so no more than a pair is live.
// After the halvings the quad's four lanes are summed (xor 1, xor 2): lane l ends with
// the full sum of row l >> 2.  Fixed order.
template <typename RowPartial>
__device__ __forceinline__ float wave_rows16(RowPartial part, int lane) {
  float v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = swap_halve<32>(part(j), part(j + 8));
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = swap_halve<16>(v[j], v[j + 4]);
  const bool h3 = (lane & 8) != 0;
#pragma unroll
  for (int j = 0; j < 2; ++j) v[j] = (h3 ? v[j + 2] : v[j]) + dpp_f32<kDppMirror>(h3 ? v[j] : v[j + 2]);
  const bool h2 = (lane & 4) != 0;
  float s = (h2 ? v[1] : v[0]) + dpp_f32<kDppHalfMirror>(h2 ? v[0] : v[1]);
  s += dpp_f32<kDppXor1>(s);
  s += dpp_f32<kDppXor2>(s);
  return s;
}

// XF (min1 only): the term as sign-bit flip, med3 and add (MAPI_MIN1_FORM=xor), the same bits.
template <int OP, bool XF = false>
__global__ void __launch_bounds__(kSmallThreads)
k_solve_small(const float* __restrict__ A, int64_t ld, int n, const float* __restrict__ w0, float* __restrict__ out,
              SolveState* __restrict__ st, int norm, int final_l2) {
  __shared__ __align__(16) float wl[2][kSmallN];
  __shared__ float yl[kSmallN];
  __shared__ int sh_done, sh_iter;
  __shared__ SolveState ss;   // the stop rule's state, advanced by thread 0
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;

  // rows kSmallRows * wave + r and columns 4 lane + e of A, zero outside n x n
  float a[kSmallRows][4];
#pragma unroll
  for (int r = 0; r < kSmallRows; ++r) {
    const int row = kSmallRows * wave + r;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int col = 4 * lane + e;
      a[r][e] = (row < n && col < n) ? A[(int64_t)row * ld + col] : 0.0f;
    }
  }
  for (int i = tid; i < kSmallN; i += kSmallThreads) {
    wl[0][i] = i < n ? w0[i] : 0.0f;
    wl[1][i] = 0.0f;
  }
  if (tid == 0) {
    ss = *st;
    sh_done = ss.done;
    sh_iter = ss.iter;
  }
  __syncthreads();

  while (!sh_done) {
    const int it = sh_iter;
    const float* w = wl[it & 1];
    const float4 wv4 = *reinterpret_cast<const float4*>(w + 4 * lane);
    const float wv[4] = {wv4.x, wv4.y, wv4.z, wv4.w};
    // min1 term as med3(a, -|w|, |w|) times s = +-1 (the sign bit of w) in one FMA: the
    // product is exact, so the term and the sum equal those of a sign flip and an add
    uint32_t ws[4];
    float sg[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      ws[e] = sign_bit(wv[e]);
      sg[e] = __uint_as_float(ws[e] | 0x3f800000u);
    }
    const float yrow = wave_rows16(
        [&](int r) {
          float t = 0.0f;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            if constexpr (OP == MAPI_OP_MIN1 && !XF)
              t = fmaf(__builtin_amdgcn_fmed3f(a[r][e], -fabsf(wv[e]), fabsf(wv[e])), sg[e], t);
            else
              t = op_acc<OP>(t, a[r][e], wv[e], ws[e]);
          }
          return t;
        },
        lane);
    const int row = kSmallRows * wave + (lane >> 2);
    if ((lane & 3) == 0 && row < n) yl[row] = yrow;
    __syncthreads();
    if (wave == 0) {
      // element i = lane + 64 q of y, w_{t-1} and the new iterate
      float yv[4], wo[4];
      double sq = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = lane + kWave * q;
        yv[q] = i < n ? yl[i] : 0.0f;
        wo[q] = w[i];
        sq += (norm == NORM_L2) ? (double)yv[q] * (double)yv[q] : fabs((double)yv[q]);
      }
      const double tot = wave_total_f64(sq);
      const double nu = (norm == NORM_L2) ? sqrt(tot) : tot;
      if (!(nu > 0.0) || !(nu < INFINITY)) {
        if (lane == 0) {
          ss.nu = nu;
          ss.status = MAPI_ERR_DEGENERATE;
          ss.done = 1;
          sh_done = 1;
        }
      } else {
        const double inv = 1.0 / nu;
        double r = 0.0;
        float* wn = wl[(it & 1) ^ 1];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = lane + kWave * q;
          const float v = (float)((double)yv[q] * inv);
          if (i < n) {
            wn[i] = v;
            r += fabs((double)v - (double)wo[q]);
          }
        }
        r = wave_total_f64(r);
        if (lane == 0) {
          ss.nu = nu;
          state_advance(&ss, r);
          sh_done = ss.done;
          sh_iter = ss.iter;
        }
      }
    }
    __syncthreads();
  }

  // the final iterate, optionally divided by its l2 norm (Algorithm 1, last step)
  const float* wf = wl[sh_iter & 1];
  __shared__ double sh[kSmallThreads / kWave];
  double scale = 1.0;
  bool write = true;
  if (final_l2) {
    const double v = tid < n ? (double)wf[tid] : 0.0;
    const double l2 = block_sum_f64(v * v, sh);
    if (!(l2 > 0.0) || !(l2 < INFINITY)) {
      write = false;
      if (tid == 0) ss.status = MAPI_ERR_DEGENERATE;
    } else {
      scale = 1.0 / sqrt(l2);
    }
  }
  if (write && tid < n) out[tid] = final_l2 ? (float)((double)wf[tid] * scale) : wf[tid];
  __syncthreads();
  if (tid == 0) *st = ss;
}

// the min forms and the ordinary product (the diamond form of eq. 7 keeps the multi-kernel path)
bool small_solve_fits(int64_t n, int op) {
  return n >= 1 && n <= kSmallN && (op == MAPI_OP_MIN1 || op == MAPI_OP_MIN2 || op == MAPI_OP_DOT);
}

hipError_t launch_solve_small(int op, const float* A, int64_t ld, int64_t n, const float* w0, float* out,
                              SolveState* st, int norm, int final_l2, hipStream_t s) {
  if (!small_solve_fits(n, op)) return hipErrorInvalidValue;
  const int ni = (int)n;
  switch (op) {
    case MAPI_OP_MIN1:
      if (min1_xor_form())
        hipLaunchKernelGGL((k_solve_small<MAPI_OP_MIN1, true>), dim3(1), dim3(kSmallThreads), 0, s, A, ld, ni, w0, out,
                           st, norm, final_l2);
      else
        hipLaunchKernelGGL(k_solve_small<MAPI_OP_MIN1>, dim3(1), dim3(kSmallThreads), 0, s, A, ld, ni, w0, out, st,
                           norm, final_l2);
      break;
    case MAPI_OP_MIN2:
      hipLaunchKernelGGL(k_solve_small<MAPI_OP_MIN2>, dim3(1), dim3(kSmallThreads), 0, s, A, ld, ni, w0, out, st, norm,
                         final_l2);
      break;
    case MAPI_OP_DOT:
      hipLaunchKernelGGL(k_solve_small<MAPI_OP_DOT>, dim3(1), dim3(kSmallThreads), 0, s, A, ld, ni, w0, out, st, norm,
                         final_l2);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mapi
