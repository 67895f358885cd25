/*
 * mapi.h -- C-ABI of libmapi.so: multiplication-avoiding power iteration (MAPI)
 * and regular power iteration (RPI) on one AMD Instinct MI355X (gfx950).
 *
 * Method: Pan, Badawi, Miao, Koyuncu, Cetin, "Multiplication-Avoiding Variant of
 * Power Iteration with Applications", arXiv 2110.12065.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers to matrices, vectors and outputs are DEVICE pointers on the
 *    context's device, owned by the caller; the library never frees them.
 *    Host pointers are only the descriptor structs, options and info outputs.
 *  - Dense matrices are row-major with a leading dimension `ld` (elements).
 *    The base pointer and the row pitch (ld * element size) must be 16-byte
 *    aligned.  Vectors must be 4-byte aligned float arrays.
 *  - Calls are blocking: work is enqueued on the context's stream and the
 *    stream is synchronised before return (mapi_mavp and mapi_quantize too).
 *  - Errors are returned as mapi_status; mapi_last_error() gives a message for
 *    the calling thread.  No C++ exception crosses this boundary.  Not reaching
 *    the tolerance is not an error: it is reported as converged = 0.
 *  - Device workspace (iteration buffers, partial sums, built matrices): by
 *    default the context allocates it on first use and keeps it until
 *    mapi_destroy.  A caller that owns its device memory (a torch tensor, say)
 *    gives the context one region with mapi_set_workspace, sized by
 *    mapi_workspace_size; every call then takes its buffers from that region
 *    and allocates no device memory (mapi_serve_* excepted: a server owns its
 *    pool).  One context must not be used from two threads at once.
 */
#ifndef MAPI_H
#define MAPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mapi_status {
  MAPI_OK = 0,
  MAPI_ERR_ARG = 1,          /* invalid argument (shape, alignment, range)        */
  MAPI_ERR_ALLOC = 2,        /* device or host allocation failed                  */
  MAPI_ERR_HIP = 3,          /* a HIP runtime call failed                          */
  MAPI_ERR_DEGENERATE = 4,   /* an iterate's normaliser was zero or not finite    */
  MAPI_ERR_BUDGET = 5,       /* request larger than the serving memory budget     */
  MAPI_ERR_UNSUPPORTED = 6,  /* combination not implemented                        */
  MAPI_ERR_PENDING = 7,      /* serving: result not ready yet                      */
  MAPI_ERR_TIMEOUT = 8,      /* serving: wait timed out                            */
  MAPI_ERR_DEVICE_CHECK = 9  /* device-checked build (libmapi_checked.so): a
                                kernel's index check failed; the message names
                                the kernel's file id and line                     */
} mapi_status;

typedef enum mapi_dtype {
  MAPI_F32 = 0,              /* IEEE binary32                                      */
  MAPI_BF16 = 1,             /* bfloat16 (upper half of binary32)                  */
  MAPI_FP8_E4M3 = 2          /* OCP FP8 E4M3 (e4m3fn) with one float32 scale per row */
} mapi_dtype;

/* The vector product that replaces the inner product (Sec. 2.1). */
typedef enum mapi_op {
  MAPI_OP_MIN1 = 0,          /* eq. (3): sum sign(a b) min(|a|, |b|)               */
  MAPI_OP_MIN2 = 1,          /* eq. (4): sum 1(sign a = sign b) min(|a|, |b|)      */
  MAPI_OP_DIAMOND = 2,       /* eq. (7): sum sign(a) b + a sign(b)                 */
  MAPI_OP_DOT = 3            /* the ordinary inner product (RPI, eq. 1)            */
} mapi_op;

typedef enum mapi_method { MAPI_METHOD_MAPI = 0, MAPI_METHOD_RPI = 1 } mapi_method;

/* Dense matrix descriptor.  row_scale: FP8 only, device float[n_rows];
 * element (i, j) is fl32(row_scale[i] * decode(data[i * ld + j])).  Any positive
 * scale is accepted; rows whose scale is a power of two (as mapi_quantize writes)
 * use the scaled-conversion decode, others a separate multiply -- same values.  */
typedef struct mapi_dense {
  const void* data;
  int64_t n_rows, n_cols, ld;
  int32_t dtype;             /* mapi_dtype */
  const float* row_scale;
} mapi_dense;

/* Link matrix H in CSR by destination row: row i lists the sources j of the
 * links j -> i with value H_ij (column-stochastic).  Column indices within a row
 * need not be sorted; a node that is never a source is dangling.               */
typedef struct mapi_csr {
  int64_t n, nnz;
  const int32_t* row_ptr;    /* device int32[n + 1], row_ptr[0] = 0, row_ptr[n] = nnz */
  const int32_t* col;        /* device int32[nnz], values in [0, n)             */
  const float* val;          /* device float[nnz]                               */
} mapi_csr;

typedef struct mapi_opts {
  int32_t max_iters;         /* T of Algorithm 1 (>= 0)                           */
  double tol;                /* stop when ||w_t - w_{t-1}||_1 < tol; 0 = run T    */
  int32_t final_l2;          /* divide the result by its l2 norm (Algorithm 1)    */
  int32_t op;                /* mapi_op for MAPI calls (ignored by RPI)           */
  int32_t check_every;       /* host polls the stop flag every k iterations (0 = 16) */
  int32_t stall_iters;       /* stop, unconverged, after this many iterations without
                                a new smallest residual (0 = never)              */
} mapi_opts;

typedef struct mapi_info {
  int32_t iters;             /* iterations run                                     */
  int32_t converged;         /* 1 if the residual fell below tol                   */
  double residual;           /* last ||w_t - w_{t-1}||_1                           */
  double norm;               /* last normaliser (l1 for MAPI / PageRank, l2 for RPI) */
  int32_t status;            /* mapi_status of this solve                          */
} mapi_info;

typedef struct mapi_ctx mapi_ctx;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t, or NULL for the default stream).                             */
mapi_status mapi_create(int device, void* hip_stream, mapi_ctx** out);
void mapi_destroy(mapi_ctx* ctx);
mapi_status mapi_set_stream(mapi_ctx* ctx, void* hip_stream);
/* Message of the last error on the calling thread ("" if none). */
const char* mapi_last_error(void);
/* Library version string. */
const char* mapi_version(void);

/* ---------------------------------------------------------------- workspace */

/* What a call keeps in device memory besides the caller's inputs and outputs,
 * sized by mapi_workspace_size(ctx, kind, n, nnz, &bytes); n and nnz per kind: */
typedef enum mapi_ws_kind {
  MAPI_WS_SOLVE = 0,         /* mapi_solve, rpi_solve: n = matrix order            */
  MAPI_WS_HYBRID = 1,        /* mapi_hybrid_solve: n = matrix order                */
  MAPI_WS_PAGERANK = 2,      /* mapi_pagerank: n = nodes, nnz = links              */
  MAPI_WS_PAGERANK_F64 = 3,  /* mapi_pagerank_f64: n = nodes, nnz = links          */
  MAPI_WS_PRODUCT = 4,       /* mapi_mavp, mapi_mavp_timed, mapi_autotune_dense,
                                mapi_read_reference: n = rows, nnz = columns
                                (n = nnz includes a solve's buffers: the
                                autotuner times square matrices on iterations) */
  MAPI_WS_MINGRAM = 5,       /* mapi_mingram: n = D, nnz = N samples               */
  MAPI_WS_PCA = 6,           /* mapi_pca_topk with k = 1: n = D, nnz = N samples;
                                each further vector adds MAPI_WS_PCA_VECTOR        */
  MAPI_WS_PCA_VECTOR = 7,    /* bytes per principal vector: n = D                  */
  MAPI_WS_IMAGE = 8,         /* mapi_image_reconstruct: n = P pixels, nnz = N images */
  MAPI_WS_MINIBATCH = 9,     /* mapi_minibatch as the context would run it: n = D,
                                nnz = runs (batch matrices of up to 256 MiB)      */
  MAPI_WS_MINIBATCH_MIN = 10,/* mapi_minibatch's least workspace (batch matrices of
                                one step of t per launch): n = D, nnz = runs      */
  MAPI_WS_FACTORED = 11      /* mapi_factored_solve: n = D, nnz = N samples        */
} mapi_ws_kind;

/* Bytes of caller workspace that any call of `kind` at that size needs (an upper
 * bound over launch shapes and products).  Host-only arithmetic, no device work;
 * MAPI_ERR_ARG for an unknown kind or sizes out of range.  Sizes depend on the
 * context's device (its compute-unit count).                                    */
mapi_status mapi_workspace_size(const mapi_ctx* ctx, int32_t kind, int64_t n, int64_t nnz, size_t* bytes);

/* Give the context a device region (on its device, 256-byte aligned, owned by the
 * caller and kept alive and unused by others while set) for all its calls: they
 * carve their buffers from its start and allocate no device memory.  A call that
 * needs more than `bytes` fails with MAPI_ERR_ARG before any device work
 * (mapi_minibatch builds fewer steps of batch matrices per launch to fit, down to
 * MAPI_WS_MINIBATCH_MIN).  Calls are blocking, so one region serves them in turn;
 * its contents are not kept between calls.  dev_ptr NULL (bytes 0) returns to
 * context-owned memory.  Synchronises the context stream and frees the device
 * memory the context had allocated for itself.                                  */
mapi_status mapi_set_workspace(mapi_ctx* ctx, void* dev_ptr, size_t bytes);

/* Kernel timing: when enabled, every launch of the kind below is bracketed by
 * HIP events on the context stream; mapi_timing_get returns the summed
 * duration in milliseconds and the number of launches since the last reset.  */
typedef enum mapi_kernel_kind {
  MAPI_K_MAVP = 0,           /* dense product kernel (MAPI and RPI); a one-block solve counts once */
  MAPI_K_FINALIZE = 1,       /* normalisation + residual kernel                */
  MAPI_K_GRAM = 2,           /* min-covariance / covariance build              */
  MAPI_K_CSR = 3,            /* PageRank product kernel                        */
  MAPI_K_DEFLATE = 4,        /* deflation kernels                              */
  MAPI_K_BATCHED = 5,        /* persistent batched kernel                      */
  MAPI_K_MINIBATCH = 6,      /* mini-batch MAPI with momentum kernel           */
  MAPI_K_KINDS = 7
} mapi_kernel_kind;
mapi_status mapi_timing_enable(mapi_ctx* ctx, int enable);
mapi_status mapi_timing_get(mapi_ctx* ctx, int kind, double* total_ms, int64_t* launches);
mapi_status mapi_timing_reset(mapi_ctx* ctx);

/* ---------------------------------------------------------------- products */

/* One product y = A (+) w, the matrix extension of the vector products of
 * eqs. (3), (4), (7) (Sec. 2.1): y_i = sum_j op(A_ij, w_j) for every row i;
 * with MAPI_OP_DOT the ordinary y = A w.  Float32 accumulation.
 * A: n_rows x n_cols (any dtype); w: device float[n_cols]; y: device float[n_rows]. */
mapi_status mapi_mavp(mapi_ctx* ctx, const mapi_dense* A, const float* w, float* y, int32_t op);

/* ---------------------------------------------------------------- launch shapes */

/* Launch shape of the dense product kernel.  Results of the product y are
 * bitwise independent of the shape; the float64 normaliser's summation order
 * depends on it, so one shape is kept per size bucket.                          */
typedef struct mapi_tuning {
  int32_t rows_per_wave;     /* 1, 2, 4 or 8 rows share each staged w value      */
  int32_t waves;             /* waves per block: 4 or 8                            */
  int32_t blocks_per_cu;     /* grid = compute units * blocks_per_cu (1..16)       */
  int32_t unroll;            /* 16-byte loads in flight per row and lane: 2 or 4   */
  int32_t w_in_lds;          /* 0: w read from global memory; 1: w staged in LDS
                                (4 * n_cols bytes per block); 2, FP8 storage only:
                                |w| and one sign word per 4 columns in LDS
                                (5 * n_cols bytes), one xor flips 4 stored values */
  int32_t nontemporal;       /* non-temporal matrix loads                          */
} mapi_tuning;

/* Autotuner (project-written): times every admissible launch shape on A with
 * product `op` and stores the fastest in the context's table for A's bucket
 * (storage type, ceil(log2 n_rows), ceil(log2 n_cols)); later products and
 * solves in that bucket use it.  A square matrix is timed on `reps` solve
 * iterations per shape, enqueued as a solve enqueues them (the six fastest are
 * timed three more times and the best of each one's timings decides); a
 * rectangular one, or one whose normaliser is zero, on `reps` bare products.
 * HIP events on the context stream.  If the environment variable
 * MAPI_TUNE_CACHE names a file, tuned entries are appended to it and read back
 * by mapi_create.  best / best_ms (optional, host) receive the choice and its
 * mean time per launch (per iteration for a square matrix).                    */
mapi_status mapi_autotune_dense(mapi_ctx* ctx, const mapi_dense* A, int32_t op, int32_t reps,
                                mapi_tuning* best, double* best_ms);
/* Read or overwrite the table entry used for a (dtype, n_rows, n_cols) bucket.
 * A bucket written by mapi_tuning_set is pinned: its solves always use the
 * per-iteration product and normalisation kernels with that shape, also where
 * the one-block solve (mapi_solve) would apply.                                  */
mapi_status mapi_tuning_get(mapi_ctx* ctx, int32_t dtype, int64_t n_rows, int64_t n_cols, mapi_tuning* out);
mapi_status mapi_tuning_set(mapi_ctx* ctx, int32_t dtype, int64_t n_rows, int64_t n_cols, const mapi_tuning* t);
/* Mean time in ms of `reps` products y = A (+) w with an explicit launch shape. */
mapi_status mapi_mavp_timed(mapi_ctx* ctx, const mapi_dense* A, const float* w, float* y, int32_t op,
                            const mapi_tuning* t, int32_t reps, double* avg_ms);
/* Bandwidth reference: mean time in ms of `reps` plain 16-byte-vector copies of
 * `bytes` (multiple of 16) from src to dst (device, 16-byte aligned).            */
mapi_status mapi_copy_reference(mapi_ctx* ctx, const void* src, void* dst, size_t bytes, int32_t reps,
                                double* avg_ms);
/* Bandwidth reference: mean time in ms of `reps` plain streaming reads of `bytes`
 * (multiple of 16) at src (device, 16-byte aligned): non-temporal 16-byte loads,
 * nothing written back; the fastest of 12 launch shapes (1..32 blocks of 256
 * threads per compute unit, four or eight loads per lane in flight), each timed
 * over `reps` reads after one untimed.  Uses 256 bytes of the context workspace. */
mapi_status mapi_read_reference(mapi_ctx* ctx, const void* src, size_t bytes, int32_t reps, double* avg_ms);

/* ---------------------------------------------------------------- solvers */

/* MAPI, eq. (6) and Algorithm 1: w <- (A (+) w) / ||A (+) w||_1 for at most
 * opts->max_iters iterations, stopping once ||w_t - w_{t-1}||_1 < opts->tol;
 * optional final l2 normalisation.  A must be square.  w0 (device float[n]) is
 * used exactly as given (the product is not homogeneous in w alone).  The
 * normaliser and the residual are accumulated in float64, the iterate is
 * float32.  w_out (device float[n]) may alias w0.  MAPI_ERR_DEGENERATE if a
 * normaliser is zero or not finite; info->iters then counts completed steps.
 * A float32 system with n <= 256, op MIN1 or MIN2 (rpi_solve: any such system)
 * and max_iters <= 65536 is solved by one launch of one block that holds A in registers and
 * runs every iteration, normalisation and stop test inside the kernel, unless
 * its bucket is pinned (mapi_tuning_set); larger systems, other storage types
 * and the diamond product launch a product and a normalisation per iteration.
 * The two paths differ only in the order of the row and norm sums.              */
mapi_status mapi_solve(mapi_ctx* ctx, const mapi_dense* A, const float* w0, float* w_out,
                       const mapi_opts* opts, mapi_info* info);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): mapi_solve with every
 * buffer of the solve (state, partial sums, two iterates, two products) in a static
 * device array of the library, 4 MiB on each device, held from the context's
 * creation on that device until the process ends.  Same arguments, checks, kernels
 * and results as mapi_solve; the caller still passes A, w0 and w_out (device).  No
 * device or host memory is allocated and no event is created (kernel timing is not
 * recorded for this call).  MAPI_ERR_ARG, before any device work, when the system
 * needs more than the array holds (mapi_workspace_size with MAPI_WS_SOLVE gives the
 * need; n up to about 250000 fits).  All calls on one device share that device's
 * array, whatever their context, and it keeps the last call's contents: calls that
 * overlap on one device (from two threads, or on two streams) race and must be
 * serialised by the caller.                                                        */
mapi_status mapi_solve_noalloc(mapi_ctx* ctx, const mapi_dense* A, const float* w0, float* w_out,
                               const mapi_opts* opts, mapi_info* info);

/* RPI, eq. (1): b <- A b / ||A b||_2 (float32 fused multiply-add products,
 * float64 norms), same stopping rule and arguments as mapi_solve (opts->op is
 * ignored).                                                                     */
mapi_status rpi_solve(mapi_ctx* ctx, const mapi_dense* A, const float* w0, float* w_out,
                      const mapi_opts* opts, mapi_info* info);

/* MAPI, then RPI from its result (Sec. 3.2: the MAPI iterate keeps the
 * eigenvector's information and ranks; to drive 1 - cos^2 to the top
 * eigenvector towards 0, optimise with MAPI first and switch to RPI).  Runs
 * mapi_solve with first_opts (final_l2 forced on: the hand-over vector has unit
 * l2 norm, kept in a context buffer), then rpi_solve from that vector with
 * then_opts into w_out.  info_mapi / info_rpi (optional, host) report each phase;
 * errors of either phase are returned as by mapi_solve and rpi_solve.          */
mapi_status mapi_hybrid_solve(mapi_ctx* ctx, const mapi_dense* A, const float* w0, float* w_out,
                              const mapi_opts* first_opts, const mapi_opts* then_opts, mapi_info* info_mapi,
                              mapi_info* info_rpi);

/* Image reconstruction via MAPI (Algorithm 2, Sec. 3.1) from N corrupted copies
 * of one image: V (device float32, P x N, row pitch ldv >= N) holds the P pixels
 * of copy i in column i.  m = mean of the columns; Vc = V - m; (+) is opts->op,
 * min1 (eq. 3) or min2 (eq. 4, Table 1's min2-PI), in every step:
 *   C  = (1/(N-1)) Vc (+) Vc^T                 (line 4; RPI: Vc Vc^T / (N-1))
 *   w1 = MAPI on C                              (line 5; RPI: eq. 1)
 *   w2 = MAPI on C - (w1 (+) w1^T) C            (line 6; RPI: C - w1 w1^T C)
 *   R  = (W (+) W^T) Vc + m, W = [w1 w2]         (line 8; RPI: W W^T Vc + m)
 * Both solves start from w0 (device, P, 16-byte aligned) and follow opts
 * (max_iters, tol, check_every, stall_iters; op MAPI_OP_MIN1 or MAPI_OP_MIN2 for
 * MAPI, else MAPI_ERR_UNSUPPORTED; final_l2 is ignored).  MAPI vectors are returned as Algorithm 1 leaves them,
 * with unit l1 norm -- the unit of the operator (w (+) w = ||w||_1, Sec. 2.1), so
 * that w (+) w^T acts on w as w w^T does for an l2 unit vector; RPI vectors have
 * unit l2 norm.  R: device P x N (pitch ldr >= N),
 * the N reconstructions; W: device P x 2 (w1 at W, w2 at W + P).  info2: host,
 * 2 entries (optional).  The min-outer deflation is computed exactly in O(P^2)
 * by prefix sums over C's rows in the order of |w1| (no P^3 product; for min2
 * kept separately over the rows of each sign of w1).  2 <= N <=
 * 16, P <= 32768; about 2 P^2 floats of workspace (MAPI_WS_IMAGE).              */
mapi_status mapi_image_reconstruct(mapi_ctx* ctx, const float* V, int64_t P, int32_t N, int64_t ldv, int32_t method,
                                   const float* w0, const mapi_opts* opts, float* R, int64_t ldr, float* W,
                                   mapi_info* info2);

/* Mini-batch MAPI with momentum (Algorithm 3, Sec. 3.2), `runs` independent runs
 * (one GPU block each).  Run r iterates T times: with the batch
 * B_t = batch_idx[(r T + t) s .. + s) of sample indices,
 *   A_t = (1/s) sum_{i in B_t} x_i (+) x_i^T          (eq. 5 on the batch)
 *   w_{t+1} = A_t (+) w_t - beta w_{t-1},  w_{-1} = 0
 *   nu = ||w_{t+1}||_1;  w_t <- w_t / nu;  w_{t+1} <- w_{t+1} / nu
 * and writes w_T (divided by its l2 norm when final_l2) to w_out + r D.
 * op MAPI_OP_MIN1 (Algorithm 3) or MAPI_OP_DOT (the same recurrence with
 * ordinary products: the stochastic power method with momentum).
 * X: device float32 N x D, samples as ROWS (Algorithm 3's layout), row pitch
 * ldx >= D elements.  batch_idx: device int32, runs * T * s entries in [0, N)
 * (the mini batches are drawn by the caller; NULL allowed when T = 0); an index outside gives
 * MAPI_ERR_ARG and is never used as an address.  w0 / w_out: device float32,
 * runs * D.  Batch sums are float64 (min1 with D * D < 256: runs of 16 exact
 * float32 terms per chain summed in float32, the runs in float64), stored
 * float32; the product float32, nu
 * float64.  D <= 64 (MAPI_ERR_UNSUPPORTED beyond).  infos (optional, host, runs
 * entries): iterations run, last nu, status; a zero or non-finite nu stops that
 * run with MAPI_ERR_DEGENERATE (also returned).  The batch matrices do not depend
 * on the iterate and are built ahead for a range of t at a time, stored float32
 * in workspace (at most 256 MiB, plus 528 bytes per run; MAPI_WS_MINIBATCH).   */
mapi_status mapi_minibatch(mapi_ctx* ctx, const float* X, int64_t N, int64_t D, int64_t ldx, const int32_t* batch_idx,
                           int32_t s, int32_t T, double beta, int32_t op, int32_t runs, const float* w0, float* w_out,
                           int32_t final_l2, mapi_info* infos);

/* ---------------------------------------------------------------- storage */

/* Convert a float32 matrix (n_rows x n_cols, leading dimension lda) to reduced
 * storage: MAPI_BF16 -> uint16 codes, nearest value, ties to even;
 * MAPI_FP8_E4M3 -> uint8 e4m3fn codes with row scale s_i the smallest power of
 * two 2^k (k >= -126) with 448 s_i >= amax_i (1 for an all-zero row), codes =
 * e4m3fn(fl32(A_ij / s_i)) nearest, ties to even (never saturating).  Power-of-two
 * scales make the dequantised value an exact product, which the product kernels
 * apply inside the scaled e4m3 conversion.  out has leading dimension ld_out (elements);
 * row_scale (device float[n_rows]) is written for FP8 and may be NULL for BF16. */
mapi_status mapi_quantize(mapi_ctx* ctx, const float* A, int64_t n_rows, int64_t n_cols, int64_t lda,
                          int32_t dtype, void* out, int64_t ld_out, float* row_scale);

/* ---------------------------------------------------------------- PCA */

/* Gram build over the rows of X (D x N, row-major, leading dimension ldx; the N
 * samples are the columns, Sec. 1): A_ij = scale * sum_k op(X_ik, X_jk).
 * op MIN1/MIN2: the min-covariance of eq. (5), on the vector ALU; op DOT: the
 * covariance of eq. (2), on the matrix cores.  Terms are summed in float32 within
 * runs of 256 samples and in float64 across runs; A is rounded to float32 once.
 * A_out: D x D float32, leading dimension lda; the full matrix is written.  The
 * build may split the samples into up to 8 (DOT) or 16 (MIN1, MIN2) chunks (a
 * function of D, N and op only) whose float64 partial tiles live in workspace
 * (MAPI_WS_MINGRAM): at most 16 * T (T + 1) / 2 * 128 KiB, T = ceil(D / 128)
 * (1.1 GB at D = 4096).                                                         */
mapi_status mapi_mingram(mapi_ctx* ctx, const float* X, int64_t D, int64_t N, int64_t ldx,
                         double scale, int32_t op, float* A_out, int64_t lda);

/* Top-k principal vectors with deflation (Sec. 1; Sec. 2.2).  method MAPI:
 * MAPI (eq. 6, product opts->op) on the min-covariance of eq. (5); method RPI:
 * RPI (eq. 1) on the covariance of eq. (2); both built from X with `scale`.
 * Vector i is extracted from (I - P P^T) A, P the l2-normalised earlier vectors,
 * orthonormalised by modified Gram-Schmidt in float64, starting from column i of
 * W0.  W0, P_out: device float, D x k, column-major (column i at offset i*D); one
 * start per vector, so that each can be chosen (one start w0 for all: pass it k
 * times).  W0 = NULL: seeded starts, vector i from the start vector that
 * mapi_generate_dense gives for seed i (w_j = -+fl32(1 / sqrt(D)), the sign the
 * top bit of splitmix64(splitmix64(i ^ 0x1B873593) + j)).
 * info_k: host array of k infos.  The built and deflated matrices (2 D^2 floats),
 * the Gram build's partial tiles (mapi_mingram) and the float64 basis are
 * workspace (MAPI_WS_PCA + (k - 1) MAPI_WS_PCA_VECTOR).                         */
mapi_status mapi_pca_topk(mapi_ctx* ctx, const float* X, int64_t D, int64_t N, int64_t ldx,
                          int32_t k, double scale, int32_t method, const float* W0,
                          float* P_out, const mapi_opts* opts, mapi_info* info_k);

/* A variant that is NOT a method of the paper, for comparison with the PCA form:
 * power iteration with the factored operator
 *   z = X^T (+) w   (z_k = sum_i op(X_ik, w_i), the columns of X against w)
 *   y = scale * (X (+) z)   (y_i = sum_k op(X_ik, z_k), the rows of X against z)
 *   w <- y / ||y||_1, residual ||w_t - w_{t-1}||_1, stop rule as mapi_solve.
 * The paper forms A = scale * X (+) X^T first (eq. 5) and iterates on A; (+) is not
 * associative, so this is a different operator.  It never forms the D x D matrix and
 * streams X twice per iteration.  X: device float32 D x N, row-major (samples as
 * columns), base and row pitch ldx 16-byte aligned.  opts->op MAPI_OP_MIN1 or
 * MAPI_OP_MIN2 (else MAPI_ERR_UNSUPPORTED); w0, w_out: device float[D] (may alias);
 * info->norm is the normaliser of y, scale included.  Float32 sums (the column sums
 * in row chunks added in a fixed order), float64 normaliser and residual.          */
mapi_status mapi_factored_solve(mapi_ctx* ctx, const float* X, int64_t D, int64_t N, int64_t ldx, double scale,
                                const float* w0, float* w_out, const mapi_opts* opts, mapi_info* info);

/* ---------------------------------------------------------------- PageRank */

/* Power iteration on G = alpha H + (1 - alpha)/n 1 (eq. 11, Sec. 3.3), H with
 * dangling columns replaced by 1/n, without forming G.  method MAPI: the min1
 * product applied to G; method RPI: the ordinary product.  Both use the l1
 * normaliser.  alpha in (0, 1).  w0: device float[n], or NULL for 1/n.         */
mapi_status mapi_pagerank(mapi_ctx* ctx, const mapi_csr* H, double alpha, int32_t method,
                          const float* w0, float* w_out, const mapi_opts* opts, mapi_info* info);

/* Layout of the PageRank product.  A graph with at least min_n nodes (default 2^20,
 * whose iterate outgrows one XCD's L2) is copied once per solve into 8 column blocks
 * of ceil(n / 8) sources, each block's links of every row contiguous (about 8 bytes
 * per link plus 9 bytes per node per block of workspace, counted by MAPI_WS_PAGERANK);
 * each product then gathers every block's iterate slice on one XCD, where it stays in
 * L2, and adds the 8 per-block row sums in block order.  Smaller graphs, graphs with a
 * row holding 255 or more links in one block, and min_n <= 0 use the plain CSR
 * product.  The two differ only in the order of the float32 (float64) row sums.      */
mapi_status mapi_pagerank_split_config(mapi_ctx* ctx, int64_t min_n);
/* When the split layout applies, the first `iters` products of a solve (default 4) use
 * the plain product and the layout is built only if the solve is still running then:
 * building it costs about as much as 6 plain products at 2^22 nodes, which a solve that
 * stops within a few iterations (MAPI PageRank, Sec. 3.3) never recovers.  iters = 0
 * builds it before the first product.  Deterministic: the products switch at that
 * iteration whatever the timing.  MAPI_ERR_ARG for iters < 0.                        */
mapi_status mapi_pagerank_split_after(mapi_ctx* ctx, int32_t iters);

/* The same with a float64 iterate: w0 / w_out are device double[n], every term and
 * row sum is float64 (the float32 iterate resolves about 6e-8 of w ~ 1/n, while the
 * ranking signal sits in the deviation from 1/n, of order in-degree / n; ties in
 * in-degree are broken below that resolution).  Twice the iterate's memory and
 * gather bytes.                                                                  */
mapi_status mapi_pagerank_f64(mapi_ctx* ctx, const mapi_csr* H, double alpha, int32_t method,
                              const double* w0, double* w_out, const mapi_opts* opts, mapi_info* info);

/* ---------------------------------------------------------------- batched */

typedef enum mapi_problem_kind {
  MAPI_PROB_DENSE = 0,       /* caller's square matrix (any storage)               */
  MAPI_PROB_CSR = 1,         /* PageRank on the caller's CSR link matrix           */
  MAPI_PROB_GENERATED = 2    /* dense matrix generated on the device from a seed   */
} mapi_problem_kind;

/* One instance of a batched solve.  Generated matrices: symmetric, entries
 * x_ij * sqrt(3) / (2^23 sqrt(n)) + sigma_i sigma_j * 6 / n with x_ij uniform
 * integers in [-2^23, 2^23) and sigma_i = +-1, both from SplitMix64 of the seed
 * (a Wigner bulk of radius 2 plus a planted spike); start vector
 * w0_i = +-1/sqrt(n) from the seed.  mapi_generate_dense writes both.           */
typedef struct mapi_problem {
  int32_t kind;              /* mapi_problem_kind                                  */
  int32_t method;            /* mapi_method                                        */
  mapi_dense A;              /* MAPI_PROB_DENSE                                    */
  mapi_csr H;                /* MAPI_PROB_CSR                                      */
  double alpha;              /* MAPI_PROB_CSR damping, in (0, 1)                   */
  int64_t gen_n;             /* MAPI_PROB_GENERATED size (<= 16384)                */
  int32_t gen_dtype;         /* MAPI_PROB_GENERATED storage: MAPI_F32 or MAPI_BF16 */
  uint64_t seed;             /* MAPI_PROB_GENERATED seed                           */
  const float* w0;           /* device start vector or NULL (CSR: 1/n; generated: from the seed) */
  float* w_out;              /* device result (n floats); batched solves only      */
  mapi_opts opts;            /* final_l2 must be 0; check_every is ignored         */
} mapi_problem;

/* Persistent batched solve (MAPI, eq. 6, or RPI, eq. 1; PageRank per eq. 11):
 * all `count` instances are iterated to their own stop rule by one persistent
 * kernel launched from a captured hipGraph; each instance's arithmetic (tile
 * shapes, reduction order) depends only on its own kind, storage and size, so
 * a result is the same alone and in any mix.  infos: host array of count.
 * The batch's device arena (instances, work queue, iterates, partials, generated
 * matrices) comes from the caller's workspace when one is set, else the context
 * allocates it and keeps it.                                                     */
mapi_status mapi_solve_batched(mapi_ctx* ctx, int32_t count, const mapi_problem* probs, mapi_info* infos);
/* Bytes of that arena for this list of problems (host arithmetic only; the
 * problems are checked as mapi_solve_batched checks them).                        */
mapi_status mapi_solve_batched_workspace_size(mapi_ctx* ctx, int32_t count, const mapi_problem* probs,
                                              size_t* bytes);
/* Persistent grid: compute units * blocks_per_cu blocks (1..8, default 2: the
 * kernel is built for two resident blocks per compute unit; more wait for a
 * resident block to exit).                                                       */
mapi_status mapi_batched_config(mapi_ctx* ctx, int32_t blocks_per_cu);
/* Product tile height (row split) used for dense instances of a storage type and
 * size bucket (ceil(log2 n)); the autotuner sets it from measurements.  Default:
 * about 1 MiB of matrix per tile, 4..1024 rows.  Every tile is one work item,
 * and items cost device-wide fences and a claim on one counter, which the chip
 * serialises, so small tiles lose throughput.  An instance that fits in one tile
 * is iterated by a single block without queue round trips.                       */
mapi_status mapi_batched_rows_set(mapi_ctx* ctx, int32_t dtype, int64_t n, int32_t rows_per_tile);
mapi_status mapi_batched_rows_get(mapi_ctx* ctx, int32_t dtype, int64_t n, int32_t* rows_per_tile);
/* Autotuner for the row split: solves `count` generated instances of size n with
 * each candidate tile height (fixed `iters` MAPI iterations) and keeps the fastest. */
mapi_status mapi_autotune_batched(mapi_ctx* ctx, int32_t dtype, int64_t n, int32_t count, int32_t iters,
                                  int32_t* best_rows, double* best_ms);
/* Materialise a generated problem: A (device float32, n x ld) and w0 (device, n). */
mapi_status mapi_generate_dense(mapi_ctx* ctx, int64_t n, uint64_t seed, float* A, int64_t ld, float* w0);

/* ---------------------------------------------------------------- serving */

typedef struct mapi_server mapi_server;

typedef struct mapi_serve_cfg {
  int32_t blocks_per_cu;     /* persistent grid (0 = 2)                            */
  int32_t max_slots;         /* concurrently admitted instances (0 = 2048)         */
  double idle_exit_ms;       /* an idle block exits after this long (0 = 20)       */
} mapi_serve_cfg;

/* A request: the problem (w_out ignored) and the host buffer that receives the
 * n-float result.  For MAPI_PROB_CSR requests row_ptr, col and val are HOST
 * pointers into PINNED memory (hipHostMalloc or equivalent): the persistent
 * kernel reads them itself at admission, copies them to the device and checks
 * them (row_ptr[0] = 0, row_ptr[n] = nnz, non-decreasing, 0 <= col < n); an
 * invalid request completes with MAPI_ERR_ARG and does not affect others.
 * Pageable CSR arrays are rejected by mapi_serve_submit with MAPI_ERR_ARG.  The
 * caller keeps the CSR arrays and host_out alive until the request completes.   */
typedef struct mapi_request {
  mapi_problem prob;
  float* host_out;
} mapi_request;

typedef struct mapi_result {
  int32_t status;            /* mapi_status of the solve                           */
  int32_t iters, converged;
  double residual, norm;
  double t_submit_ms, t_admit_ms, t_done_ms;   /* host clock, ms since server creation */
} mapi_result;

typedef struct mapi_serve_summary {
  int64_t submitted, admitted, completed, rejected;
  double solves_per_s;       /* completed / (last completion - first submission)   */
  double p50_ms, p99_ms;     /* submission -> result in host memory                */
  size_t budget_bytes, peak_bytes;
  int64_t kernel_launches;   /* persistent-kernel graph launches                   */
} mapi_serve_summary;

/* Continuous-batching server on `device`: admits requests while a device memory
 * budget of hbm_budget bytes (matrix, iterates, partials, CSR copy), an instance
 * slot and room for the result in a pinned output pool (min(budget, 1 GiB)) are
 * free; admitted requests join the running persistent kernel through a host
 * memory inbox, so work of requests arriving at different times overlaps on the
 * device.  Admission and completion issue no copy command or kernel (the kernel
 * reads descriptors and CSR arrays from pinned host memory and writes results
 * there), so they never wait behind the persistent kernel on a shared hardware
 * queue.  The server owns its memory and threads.                               */
mapi_status mapi_serve_create(int device, size_t hbm_budget, const mapi_serve_cfg* cfg, mapi_server** out);
/* Non-blocking: queue a request, returns its ticket.  MAPI_ERR_BUDGET (at once)
 * if its footprint alone exceeds the budget.                                     */
mapi_status mapi_serve_submit(mapi_server* s, const mapi_request* req, uint64_t* ticket);
/* MAPI_ERR_PENDING until the result is in host memory. */
mapi_status mapi_serve_poll(mapi_server* s, uint64_t ticket, mapi_result* res);
/* Block up to timeout_us (< 0: forever); MAPI_ERR_TIMEOUT if not done. */
mapi_status mapi_serve_wait(mapi_server* s, uint64_t ticket, int64_t timeout_us, mapi_result* res);
mapi_status mapi_serve_stats(mapi_server* s, mapi_serve_summary* out);
/* Waits for admitted work, stops the threads and frees everything. */
void mapi_serve_destroy(mapi_server* s);

#ifdef __cplusplus
}
#endif
#endif /* MAPI_H */
