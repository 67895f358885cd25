// Persistent batched solver: instance descriptors, the device work queue and
// the control block shared by the persistent kernel and the host runtime.
//
// Work is a stream of items (instance, phase, tile).  Blocks of the persistent
// kernel take tickets (positions) of a multi-producer multi-consumer ring in
// device memory with one fetch-add each, wait for the item of their position,
// run it, and the block that finishes the last tile of a phase pushes the next
// phase's tiles.  A block that leaves while its position is still empty marks
// the position skipped, and a producer that finds its position skipped takes a
// new one, so no item is stranded whatever the number of resident blocks.
// Items never wait on other items.  Every wait has a wall-clock limit.
#pragma once

#include "common.h"

namespace mapi {

enum BKind { BK_DENSE = 0, BK_CSR = 1, BK_GEN = 2 };
// ADMIT copies a served request's descriptor from host memory to the device;
// PREPA / PREPB copy and check a served PageRank request's CSR arrays (rows, then
// links) from pinned host memory and flag its dangling nodes.
enum BPhase {
  PH_GEN = 0, PH_INIT = 1, PH_PROD = 2, PH_FIN = 3, PH_OUT = 4,
  PH_ADMIT = 5, PH_PREPA = 6, PH_PREPB = 7, PH_SKIP = 15
};

constexpr int kVecTile = 8192;      // elements per INIT / FIN / OUT / PREPA tile
constexpr int kEdgeTile = 65536;    // links per PREPB tile
constexpr int kGenRows = 32;        // rows per generation tile
constexpr int kSoloBurst = 16;      // iterations a solo block runs before yielding
constexpr int kBatchLdsFloats = 8192;   // w staged in LDS up to this many columns
constexpr int kMaxTileRows = 1024;      // default row-split limit

struct BInst {
  // ---- description (written by the host)
  int32_t kind, method, op, dtype;
  int32_t n;
  int32_t rows_per_tile;     // product tile height
  int32_t ntiles;            // product tiles per iteration
  int32_t vtiles;            // INIT / FIN / OUT tiles
  int32_t gtiles;            // generation tiles (BK_GEN)
  int32_t solo;              // one product tile: whole iterations inside one block
  int32_t max_iters, stall_iters;
  double tol;
  int64_t ld;                // elements
  const void* A;             // BK_DENSE: caller's matrix; BK_GEN: generated into workspace
  const float* row_scale;
  const int32_t* row_ptr;
  const int32_t* col;
  const float* val;
  const uint8_t* dangling;
  float alpha, c;
  double inv_n;
  uint64_t seed;             // BK_GEN and generated start vectors
  float gen_scale, gen_spike, gen_w0;   // generator constants, rounded on the host (GenConsts)
  const float* w0;           // NULL: generated (BK_GEN) or uniform (BK_CSR)
  float* wb0;
  float* wb1;
  float* y;
  double* part;              // ntiles + 3 * vtiles doubles
  float* out;                // result (device or host-mapped)
  int32_t slot_gen;          // reuse generation of this slot (serving)
  int32_t etiles;            // PREPB tiles
  // served PageRank request: the caller's pinned host arrays (device-accessible
  // addresses), copied into row_ptr / col / val by the PREP phases; NULL otherwise
  const int32_t* src_row_ptr;
  const int32_t* src_col;
  const float* src_val;
  int64_t nnz;
  uint32_t prep_err;         // PREP checks: 1 row_ptr ends, 2 row_ptr order, 4 column out of range
  uint32_t pad0;
  // ---- dynamic state
  SolveState st;
  uint32_t arrive;           // tiles finished in the current phase
  uint32_t pad1;
  int64_t t_admit, t_start, t_done;   // wall clock (device realtime counter) of the life cycle
};

struct BQueue {
  unsigned long long head;   // next position to consume
  unsigned long long tail;   // next position to reserve for producing
  unsigned long long* item;  // cap slots (item | position tag)
  uint32_t mask;             // cap - 1, cap a power of two, at most 2^24
  uint32_t live;             // instances admitted and not finished
  uint32_t error;            // bit 0: blocks stopped at the run limit with work left
  uint32_t pad;
};

// Completion record written to host-visible memory when an instance finishes.
struct BDone {
  int32_t slot, slot_gen, status, iters, converged, pad;
  double residual, norm;
  int64_t t_admit, t_start, t_done;
  unsigned long long seq;    // written last: position + 1
};

struct BCtl {
  int32_t mode;              // 0: batch, exit when live == 0; 1: serving, exit on quit or idle
  int32_t pad;
  int64_t run_limit;         // realtime ticks after its start at which a block stops taking items
  int64_t idle_limit;        // realtime ticks a block waits for an item before it exits
  // serving inbox: host-written ring of items in host memory, drained by block 0
  const unsigned long long* inbox;       // host-mapped
  const volatile unsigned long long* inbox_tail;   // host-mapped, written by the host
  volatile unsigned long long* inbox_head_host;    // host-mapped, written by block 0
  unsigned long long inbox_head;         // device copy
  uint32_t inbox_mask;
  uint32_t pad2;
  const volatile int32_t* quit;          // host-mapped
  // completion ring in host memory
  BDone* done;                           // host-mapped
  const BInst* inst_stage;               // host-mapped descriptors written at admission (serving)
  unsigned long long done_pos;           // device counter
  uint32_t done_mask;
  uint32_t pad3;
};

// Work item: instance (20 bits), phase (4 bits), tile (15 bits).  A ring slot holds
// the item and, in its top 25 bits, the low bits of (position + 1), so a consumer
// recognises the item of the position it claims from one 64-bit load.
constexpr int kTagShift = 39;
constexpr unsigned long long kItemMask = (1ull << kTagShift) - 1;
constexpr uint32_t kMaxInstances = 1u << 20;
constexpr uint32_t kMaxTiles = 32767;
__host__ __device__ inline unsigned long long bitem(uint32_t inst, int phase, uint32_t tile) {
  return (unsigned long long)inst | ((unsigned long long)phase << 20) | ((unsigned long long)tile << 24);
}
__host__ __device__ inline unsigned long long bslot(unsigned long long pos, unsigned long long item) {
  return item | (((pos + 1) & 0x1FFFFFFull) << kTagShift);
}
__host__ __device__ inline uint32_t item_inst(unsigned long long v) { return (uint32_t)(v & 0xFFFFFull); }
__host__ __device__ inline int item_phase(unsigned long long v) { return (int)((v >> 20) & 0xFull); }
__host__ __device__ inline uint32_t item_tile(unsigned long long v) { return (uint32_t)((v >> 24) & 0x7FFFull); }

// SplitMix64 output function (Steele, Lea and Flood, 2014), used as a
// counter-based generator: value = splitmix64(splitmix64(seed) + counter).
__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// Generated symmetric matrix: a_ij = x_ij * s_n + sigma_i sigma_j * theta / n with
// x_ij the top 24 bits of splitmix64(splitmix64(seed) + (min(i,j) << 32 | max(i,j)))
// minus 2^23 (uniform integers), s_n = fl32(sqrt(3) / (2^23 sqrt(n))) (unit-variance
// entries over sqrt(n): semicircle bulk of radius 2), theta = 6 and sigma_i the top
// bit of splitmix64(splitmix64(seed ^ 0x5BD1E995) + i) as a sign.  Rounded in float32,
// product then sum.  `same` is sigma_i == sigma_j.
__device__ __forceinline__ float gen_value(uint64_t base, int i, int j, float s_n, float spike, bool same) {
#pragma clang fp contract(off)
  const uint64_t lo = (uint64_t)min(i, j), hi = (uint64_t)max(i, j);
  const uint64_t h = splitmix64(base + ((lo << 32) | hi));
  const float x = (float)((int32_t)(h >> 40) - 8388608);
  const float prod = x * s_n;          // rounded on its own: no fused multiply-add here
  return prod + (same ? spike : -spike);
}
__device__ __forceinline__ bool gen_sign(uint64_t sbase, int i) {
  return (splitmix64(sbase + (uint64_t)i) >> 63) != 0;
}

// Rows r0 .. r1-1 (r1 - r0 <= 32) of the generated matrix, all n columns, written
// to A (row pitch ld) as float32 or, with BF16 set, rounded to nearest even
// bfloat16.  The signs are hashed once each: a row's by one lane of every wave
// (gathered by a ballot), a column's once per thread before its rows, so an entry
// costs one hash.  Every thread of the block calls it.
template <bool BF16>
__device__ __forceinline__ void gen_rows(void* A, int64_t ld, int n, int r0, int r1, uint64_t base, uint64_t sbase,
                                         float s_n, float spike) {
  const int lane = threadIdx.x & 63;
  const bool mine = lane < r1 - r0 && gen_sign(sbase, r0 + lane);
  const uint64_t rows = __ballot(mine);
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const bool sj = gen_sign(sbase, j);
    for (int i = r0; i < r1; ++i) {
      const float a = gen_value(base, i, j, s_n, spike, ((rows >> (i - r0)) & 1ull) == (uint64_t)sj);
      if (BF16) {
        uint32_t u = __float_as_uint(a);
        u += 0x7FFFu + ((u >> 16) & 1u);
        reinterpret_cast<uint16_t*>(A)[(int64_t)i * ld + j] = (uint16_t)(u >> 16);
      } else {
        reinterpret_cast<float*>(A)[(int64_t)i * ld + j] = a;
      }
    }
  }
}

hipError_t launch_persistent(BQueue* q, BInst* inst, BCtl* ctl, int blocks, hipStream_t s);

// Generator constants, computed on the host in float64 with correctly rounded
// sqrt and division and rounded once to float32.
struct GenConsts {
  float scale, spike, w0;
};
inline GenConsts gen_consts(int64_t n) {
  const double rn = __builtin_sqrt((double)n);
  return GenConsts{(float)(1.7320508075688772 / (8388608.0 * rn)), (float)(6.0 / (double)n), (float)(1.0 / rn)};
}

// host helpers shared by the batched solve and the server (batch.hip)
}  // namespace mapi
struct mapi_ctx;
namespace mapi {
mapi_status describe(mapi_ctx* c, const mapi_problem& p, BInst* I, int64_t* matrix_bytes);
size_t instance_bytes(const BInst& I, int64_t matrix_bytes);
char* place(BInst* I, char* base, int64_t matrix_bytes);
uint32_t first_phase_tiles(const BInst& I, int* phase);
uint32_t max_tiles(const BInst& I);
int64_t realtime_hz();
int persistent_threads();
hipError_t launch_gen_dense(int n, uint64_t seed, float* A, int64_t ld, float* w0, hipStream_t s);

}  // namespace mapi
