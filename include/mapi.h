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
 *  - The context allocates its own device workspace (iteration buffers, partial
 *    sums) on first use and keeps it until mapi_destroy.  One context must not
 *    be used from two threads at once.
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
  MAPI_ERR_TIMEOUT = 8       /* serving: wait timed out                            */
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
 * element (i, j) is row_scale[i] * decode(data[i * ld + j]).                   */
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

/* Kernel timing: when enabled, every launch of the kind below is bracketed by
 * HIP events on the context stream; mapi_timing_get returns the summed
 * duration in milliseconds and the number of launches since the last reset.  */
typedef enum mapi_kernel_kind {
  MAPI_K_MAVP = 0,           /* dense product kernel (MAPI and RPI)            */
  MAPI_K_FINALIZE = 1,       /* normalisation + residual kernel                */
  MAPI_K_GRAM = 2,           /* min-covariance / covariance build              */
  MAPI_K_CSR = 3,            /* PageRank product kernel                        */
  MAPI_K_DEFLATE = 4,        /* deflation kernels                              */
  MAPI_K_BATCHED = 5,        /* persistent batched kernel                      */
  MAPI_K_KINDS = 6
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
  int32_t w_in_lds;          /* stage w in LDS (needs 4 * n_cols bytes per block)  */
  int32_t nontemporal;       /* non-temporal matrix loads                          */
} mapi_tuning;

/* Autotuner (project-written): times every admissible launch shape on A with
 * product `op` (`reps` launches each, HIP events on the context stream) and
 * stores the fastest in the context's table for A's bucket (storage type,
 * ceil(log2 n_rows), ceil(log2 n_cols)); later products and solves in that
 * bucket use it.  If the environment variable MAPI_TUNE_CACHE names a file,
 * tuned entries are appended to it and read back by mapi_create.
 * best / best_ms (optional, host) receive the choice and its mean time.        */
mapi_status mapi_autotune_dense(mapi_ctx* ctx, const mapi_dense* A, int32_t op, int32_t reps,
                                mapi_tuning* best, double* best_ms);
/* Read or overwrite the table entry used for a (dtype, n_rows, n_cols) bucket. */
mapi_status mapi_tuning_get(mapi_ctx* ctx, int32_t dtype, int64_t n_rows, int64_t n_cols, mapi_tuning* out);
mapi_status mapi_tuning_set(mapi_ctx* ctx, int32_t dtype, int64_t n_rows, int64_t n_cols, const mapi_tuning* t);
/* Mean time in ms of `reps` products y = A (+) w with an explicit launch shape. */
mapi_status mapi_mavp_timed(mapi_ctx* ctx, const mapi_dense* A, const float* w, float* y, int32_t op,
                            const mapi_tuning* t, int32_t reps, double* avg_ms);
/* Bandwidth reference: mean time in ms of `reps` plain 16-byte-vector copies of
 * `bytes` (multiple of 16) from src to dst (device, 16-byte aligned).            */
mapi_status mapi_copy_reference(mapi_ctx* ctx, const void* src, void* dst, size_t bytes, int32_t reps,
                                double* avg_ms);

/* ---------------------------------------------------------------- solvers */

/* MAPI, eq. (6) and Algorithm 1: w <- (A (+) w) / ||A (+) w||_1 for at most
 * opts->max_iters iterations, stopping once ||w_t - w_{t-1}||_1 < opts->tol;
 * optional final l2 normalisation.  A must be square.  w0 (device float[n]) is
 * used exactly as given (the product is not homogeneous in w alone).  The
 * normaliser and the residual are accumulated in float64, the iterate is
 * float32.  w_out (device float[n]) may alias w0.  MAPI_ERR_DEGENERATE if a
 * normaliser is zero or not finite; info->iters then counts completed steps.  */
mapi_status mapi_solve(mapi_ctx* ctx, const mapi_dense* A, const float* w0, float* w_out,
                       const mapi_opts* opts, mapi_info* info);

/* RPI, eq. (1): b <- A b / ||A b||_2 (float32 fused multiply-add products,
 * float64 norms), same stopping rule and arguments as mapi_solve (opts->op is
 * ignored).                                                                     */
mapi_status rpi_solve(mapi_ctx* ctx, const mapi_dense* A, const float* w0, float* w_out,
                      const mapi_opts* opts, mapi_info* info);

/* ---------------------------------------------------------------- storage */

/* Convert a float32 matrix (n_rows x n_cols, leading dimension lda) to reduced
 * storage: MAPI_BF16 -> uint16 codes, nearest value, ties to even;
 * MAPI_FP8_E4M3 -> uint8 e4m3fn codes with row scale s_i = fl32(amax_i / 448)
 * (1 for an all-zero row), codes = e4m3fn(fl32(A_ij / s_i)) nearest, ties to
 * even, saturating at 448.  out has leading dimension ld_out (elements);
 * row_scale (device float[n_rows]) is written for FP8 and may be NULL for BF16. */
mapi_status mapi_quantize(mapi_ctx* ctx, const float* A, int64_t n_rows, int64_t n_cols, int64_t lda,
                          int32_t dtype, void* out, int64_t ld_out, float* row_scale);

/* ---------------------------------------------------------------- PCA */

/* Gram build over the rows of X (D x N, row-major, leading dimension ldx; the N
 * samples are the columns, Sec. 1): A_ij = scale * sum_k op(X_ik, X_jk).
 * op MIN1/MIN2: the min-covariance of eq. (5); op DOT: the covariance of eq. (2).
 * A_out: D x D float32, leading dimension lda; the full matrix is written.       */
mapi_status mapi_mingram(mapi_ctx* ctx, const float* X, int64_t D, int64_t N, int64_t ldx,
                         double scale, int32_t op, float* A_out, int64_t lda);

/* Top-k principal vectors with deflation (Sec. 1; Sec. 2.2).  method MAPI:
 * MAPI (eq. 6, product opts->op) on the min-covariance of eq. (5); method RPI:
 * RPI (eq. 1) on the covariance of eq. (2); both built from X with `scale`.
 * Vector i is extracted from (I - P P^T) A, P the l2-normalised earlier vectors,
 * orthonormalised by modified Gram-Schmidt in float64, starting from column i of
 * W0.  W0, P_out: device float, D x k, column-major (column i at offset i*D).
 * info_k: host array of k infos.  If A_ws is non-NULL it must hold D*D floats of
 * device scratch for the built matrix (else the context allocates it).          */
mapi_status mapi_pca_topk(mapi_ctx* ctx, const float* X, int64_t D, int64_t N, int64_t ldx,
                          int32_t k, double scale, int32_t method, const float* W0,
                          float* P_out, const mapi_opts* opts, mapi_info* info_k);

/* ---------------------------------------------------------------- PageRank */

/* Power iteration on G = alpha H + (1 - alpha)/n 1 (eq. 11, Sec. 3.3), H with
 * dangling columns replaced by 1/n, without forming G.  method MAPI: the min1
 * product applied to G; method RPI: the ordinary product.  Both use the l1
 * normaliser.  alpha in (0, 1).  w0: device float[n], or NULL for 1/n.         */
mapi_status mapi_pagerank(mapi_ctx* ctx, const mapi_csr* H, double alpha, int32_t method,
                          const float* w0, float* w_out, const mapi_opts* opts, mapi_info* info);

#ifdef __cplusplus
}
#endif
#endif /* MAPI_H */
