/*
 * gj.h -- C ABI of libgj: Gauss-Jordan matrix inversion with full pivoting on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: C. V. Anghel Drugarin, "Numerical application and Turbo C program
 * using the Gauss-Jordan method" (arXiv:1401.7962), section 2:
 *   - A^0 = A, D^0 = I (eqs. 1-2); n steps; A^n = I and A^-1 = D^n (eqs. 11-12);
 *   - at each step the element of largest |a| in the trailing block is brought
 *     to the pivot position by swapping rows k,i and columns k,j (Obs. 2-3);
 *   - the pivot rows of A and D are divided by the pivot (eq. 14) and every
 *     other row i receives -a_ik times the new pivot row (eq. 15);
 *   - det A is the product of the pivots (eq. 13);
 *   - a pivot that is null or below a preset zero threshold, with no other
 *     candidate left, means A is singular (Obs. 2);
 *   - the swaps are undone in reverse order at the end (Obs. 3, conclusions).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array argument is a DEVICE pointer owned by the caller.  The
 *   library allocates nothing per call and keeps no pointer after the work it
 *   enqueued has finished.  Scratch space is the caller's workspace `ws` of
 *   `ws_bytes` bytes (at least gj_workspace_size(...), 256-byte aligned).
 * Layout.  Row-major, leading dimension >= n, in elements.  A is never
 *   written; X must not overlap A or the workspace.
 * Stream.  `stream` is a hipStream_t (NULL = the null stream).  Every call
 *   enqueues its kernels on it and returns; results are valid once the stream
 *   has been synchronised.  Outside graph capture, the refined single-matrix
 *   path (gj_invert, gj_det with GJ_PREC_FP32_REFINED) enqueues its FP64
 *   fallback on a second stream of the device that the library creates once,
 *   and makes `stream` wait for it before the call's last work: synchronising
 *   `stream` still covers everything.  gj_invert_batched (plain FP64) runs its
 *   one-matrix-per-wavefront classes on that same stream, also under graph
 *   capture once an earlier call outside capture has created it, and joins it
 *   back the same way.  The return value covers only argument checks and
 *   launch errors; numeric outcomes (singular, non-finite) are reported per
 *   matrix in the device-side gj_result.
 * Pivots.  0-based, LAPACK xGETC2 convention: at step k rows k <-> ipiv[k] and
 *   columns k <-> jpiv[k] of the current (already swapped) matrix were
 *   exchanged.  Ties between equal |a| go to the lowest row, then the lowest
 *   column, of the current matrix.  Steps not taken hold -1.
 * Determinant.  Kept exactly as det_sign * det_mant * 2^det_exp with det_mant
 *   in [0.5, 1): the product of pivots in step order, renormalised after every
 *   multiplication, so it neither overflows nor underflows.
 * Errors.  No C++ exception crosses this boundary.  A singular matrix is not an
 *   error: the call returns GJ_OK and the matrix's gj_result says SINGULAR.
 * Threads.  Library state is read-only after load, apart from a mutex-guarded
 *   record of the batched plans uploaded into each workspace (for
 *   GJ_FLAG_REUSE_PLAN), the per-device address of gj_invert_noalloc's array
 *   and the per-device second stream; calls on different streams with
 *   different workspaces may run concurrently.
 */
#ifndef GJ_H
#define GJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes of the entry points (synchronous checks and launches). */
typedef enum {
    GJ_OK = 0,
    GJ_E_INVALID_ARG = -1,  /* n < 1, ld < n, NULL pointer, overlap, bad option */
    GJ_E_WORKSPACE = -2,    /* ws_bytes smaller than gj_workspace_size() or misaligned */
    GJ_E_HIP = -3,          /* a HIP runtime call or launch failed */
    GJ_E_UNSUPPORTED = -4   /* size or option combination the library does not handle */
} gj_status;

/* Per-matrix outcome (gj_result.code). */
enum {
    GJ_RES_OK = 0,
    GJ_RES_SINGULAR = 1,        /* every candidate pivot was 0 or below the zero threshold */
    GJ_RES_NONFINITE = 2,       /* a NaN or infinity appeared among the candidates */
    GJ_RES_REFINE_FALLBACK = 3  /* refined path: refinement did not converge; the plain
                                   FP64 elimination produced the result instead */
};

/* gj_opts.precision */
enum {
    GJ_PREC_FP64 = 0,          /* FP64 elimination; bit-exact with the reference order */
    GJ_PREC_FP32_REFINED = 1   /* FP32 elimination, FP64 Newton-Schulz refinement
                                  X <- X + X (I - A X), FP64 determinant */
};

/* gj_opts.flags */
enum {
    GJ_FLAG_REUSE_PLAN = 1,   /* gj_invert_batched: the workspace already holds the plan that
                                 an earlier call uploaded; skip the upload (and the stream
                                 synchronisation it needs), e.g. while capturing a HIP graph.
                                 The uploaded tables hold the buffers' addresses, so the call
                                 must repeat that upload's n_host / off_host / piv_off_host,
                                 A, X, ipiv, jpiv, res, precision, workspace and ws_bytes;
                                 otherwise it returns GJ_E_INVALID_ARG and launches nothing
                                 (the library keeps a signature of the last upload into each
                                 of the 64 most recently used workspaces) */
    GJ_FLAG_PIVOT_PARTIAL = 2, /* gj_invert, gj_det, gj_solve (FP64): partial pivoting on |a|
                                 instead of the full search of Obs. 2-3: at step k the largest
                                 |a| in column k, first row wins; rows swapped, columns never
                                 (jpiv[k] = k) */
    GJ_FLAG_PIVOT_PROGRAM = 4, /* as GJ_FLAG_PIVOT_PARTIAL, but with the rule of the program in
                                 section 3: the row with the largest value greater than 0 in
                                 column k, else row k itself (its pivot may then be zero or
                                 negative).  With either rule a zero_tol < 0 means no preset
                                 threshold (the program has none): only a zero pivot is
                                 singular.  Not both; not with GJ_PREC_FP32_REFINED or
                                 gj_invert_batched (GJ_E_UNSUPPORTED).  Every order then goes
                                 through the streaming kernels. */
    GJ_FLAG_ACCURATE = 8,     /* GJ_PREC_FP32_REFINED only (else GJ_E_INVALID_ARG), gj_invert
                                 (gj_invert_batched: GJ_E_UNSUPPORTED): after the FP64
                                 Newton-Schulz loop, up to 2 more updates with residuals
                                 I - A X formed from error-free split products on the FP64
                                 matrix cores, while ||I - A X||_F at least halves.  The FP64
                                 residual stalls at about n u cond(A); these bring the forward
                                 error of X to about u.  gj_result.refine_iters counts all
                                 updates kept.  The workspace grows by 6 n^2 doubles. */
    GJ_FLAG_BLOCKED = 16      /* gj_invert with the full search only (else GJ_E_INVALID_ARG;
                                 gj_det, gj_solve, gj_invert_batched: GJ_E_UNSUPPORTED): delayed
                                 updates.  Each step eliminates on the trailing block of rows and
                                 columns not yet pivoted (all that the full search of Obs. 2-3
                                 reads); every 256 steps the other rows and columns receive those
                                 steps' eqs. 14-15 at once as matrix-core products (the theorem
                                 of section 1: the left factors of the elimination may be
                                 grouped).  GJ_PREC_FP64: pivots, rank, result code and
                                 determinant are bit-identical to the unblocked elimination; the
                                 inverse agrees up to rounding (the products sum in another
                                 order), not bit for bit.  GJ_PREC_FP32_REFINED: the FP32 stage
                                 runs this way (FP32 products), with the unblocked FP32 stage's
                                 pivots; refinement, fallback and determinant follow as without
                                 the flag.  Orders up to 128 run the on-chip kernel as without
                                 the flag.  The workspace holds two n x (n + padding) arrays of
                                 the elimination's precision.  step_events (FP64) are not
                                 recorded. */
};

/* gj_workspace_size op codes */
enum { GJ_OP_INVERT = 0, GJ_OP_DET = 1, GJ_OP_INVERT_BATCHED = 2, GJ_OP_SOLVE = 3 };

/* Per-matrix result, written to device memory by every entry point. */
typedef struct gj_result {
    int32_t code;          /* GJ_RES_* */
    int32_t rank;          /* pivot steps completed (n when OK) */
    int32_t det_sign;      /* -1 or +1; 0 when singular or non-finite */
    int32_t refine_iters;  /* Newton-Schulz updates applied (refined path), else 0 */
    double det_mant;       /* |det| = det_mant * 2^det_exp, det_mant in [0.5, 1) */
    int64_t det_exp;
    double det;            /* det as a double (may overflow to +-inf or underflow to 0) */
    double logabsdet;      /* ln|det| (-inf when singular) */
    double resid;          /* ||A X - I||_F / (||A||_F ||X||_F) if requested, else NaN */
} gj_result;

/* Options; pass NULL for the defaults shown. */
typedef struct gj_opts {
    int32_t precision;        /* GJ_PREC_FP64 */
    int32_t want_resid;       /* 0; 1 = compute gj_result.resid (one extra FP64 product) */
    int32_t max_refine_iters; /* 10; refined path: at most this many Newton-Schulz updates */
    int32_t flags;            /* 0; GJ_FLAG_* bits */
    double zero_tol;          /* -1; < 0 selects tau = n * 2^-52 * max|a_ij| (FP64
                                 elimination) and tau = 0 (FP32 elimination); >= 0 is
                                 used as given.  A step is singular when its best
                                 candidate m satisfies m == 0 or m < tau (Obs. 2). */
    void *step_events[2];     /* NULL; optional hipEvent_t pair recorded on `stream`
                                 just before the first and just after the last
                                 elimination-step kernel (used for timing) */
} gj_opts;

/*
 * gj_invert -- inverse, determinant and pivot sequence of one n x n matrix.
 *   n          order, 1 <= n <= 16384
 *   A, lda     input matrix (FP64), read only
 *   X, ldx     output inverse (FP64); all NaN when the matrix is singular or
 *              non-finite
 *   ipiv, jpiv n int32 each: the pivot sequence (see Pivots above)
 *   res        one gj_result
 *   opts       NULL or options
 *   ws         workspace of gj_workspace_size(GJ_OP_INVERT, n, NULL, opts) bytes
 * Paper: eqs. 1-2, 11-15, Obs. 2-3.
 */
gj_status gj_invert(int32_t n, const double *A, int64_t lda, double *X, int64_t ldx,
                    int32_t *ipiv, int32_t *jpiv, gj_result *res, const gj_opts *opts,
                    void *ws, size_t ws_bytes, void *stream);

/*
 * gj_invert_batched -- many independent matrices of uneven order in one call.
 *   batch          number of matrices (>= 1)
 *   n_host         HOST array [batch]: order of each matrix (1..16384)
 *   off_host       HOST array [batch]: element offset of matrix b in A and in X;
 *                  matrix b is A + off_host[b], row-major with ld = n_host[b]
 *   A, X           packed device buffers (FP64); X regions must not overlap A
 *   piv_off_host   HOST array [batch]: element offset of matrix b's pivots in
 *                  ipiv / jpiv (n_host[b] entries each)
 *   res            device array [batch] of gj_result
 *   ws             workspace of gj_workspace_size(GJ_OP_INVERT_BATCHED, batch,
 *                  n_host, opts) bytes
 * The host arrays are read during the call only.  Matrices up to the on-chip
 * limit are inverted one per workgroup (or one per wavefront) by persistent
 * launches, one per size class, that take them from atomic queues, largest
 * first (the one-per-wavefront classes on the second stream described under
 * Stream); larger ones go through the streaming path, grouped by the number
 * of register chunks their rows fill, one launch per elimination step for
 * each group, the groups one after another.  Matrices A and X are checked for overlap with each other
 * and with the workspace over the span the members cover.
 * Paper: as gj_invert, applied to each matrix.
 */
gj_status gj_invert_batched(int32_t batch, const int32_t *n_host, const int64_t *off_host,
                            const double *A, double *X, const int64_t *piv_off_host,
                            int32_t *ipiv, int32_t *jpiv, gj_result *res,
                            const gj_opts *opts, void *ws, size_t ws_bytes, void *stream);

/*
 * gj_invert_noalloc -- gj_invert for callers that cannot allocate memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same inversion with the same results, bit for bit, but
 * with no workspace argument.  Its kernels use a scratch array built into
 * the library (GJ_NOALLOC_SCRATCH_BYTES bytes, 256-byte aligned), which every
 * GPU the library runs on holds from module load until the process ends.
 * The call allocates nothing: no hipMalloc, hipFree or allocating library
 * routine.
 *   Arguments as for gj_invert, without ws / ws_bytes.  `stream` must belong
 *   to the calling thread's current device (else GJ_E_INVALID_ARG).
 *   Returns GJ_E_UNSUPPORTED when the workspace the call needs,
 *   gj_workspace_size(GJ_OP_INVERT, n, NULL, opts), exceeds
 *   GJ_NOALLOC_SCRATCH_BYTES (plain FP64: up to n = 2800 or so).
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (the kernels initialise what they read).  Calls that overlap in
 * time on one GPU -- on different streams, or from different threads --
 * race on the array: serialise them.
 */
#define GJ_NOALLOC_SCRATCH_BYTES (64u << 20)
gj_status gj_invert_noalloc(int32_t n, const double *A, int64_t lda, double *X, int64_t ldx,
                            int32_t *ipiv, int32_t *jpiv, gj_result *res, const gj_opts *opts,
                            void *stream);

/*
 * gj_det -- determinant and pivot sequence only.  Runs the same elimination
 * restricted to the rows still to be pivoted; the trailing-block values are
 * produced by the identical operations, so the pivots and the determinant
 * equal those of gj_invert bit for bit.  The inverse is not formed.
 * Paper: eq. 13 and the conclusions (the determinant at no extra cost).
 */
gj_status gj_det(int32_t n, const double *A, int64_t lda, int32_t *ipiv, int32_t *jpiv,
                 gj_result *res, const gj_opts *opts, void *ws, size_t ws_bytes,
                 void *stream);

/*
 * gj_solve -- X = A^-1 B for one n x n matrix and m right-hand sides.  Runs
 * the elimination of gj_invert on the augmented array [A | B] (eq. 2 with
 * D^0 = B in place of I; eqs. 14-15 update both parts; B's columns are never
 * pivot candidates), so the pivot sequence and the determinant equal those
 * of gj_invert bit for bit.  The column swaps of A come back as row swaps of
 * the result (Obs. 3).
 *   n          order, 1 <= n, and n + m <= 16384
 *   m          number of right-hand sides, >= 1
 *   A, lda     input matrix (FP64, row-major), read only
 *   B, ldb     right-hand sides (n x m, FP64, row-major), read only
 *   X, ldx     output (n x m, FP64); must overlap neither A, B nor ws; all NaN
 *              when the matrix is singular or non-finite
 *   ipiv, jpiv n int32 each: the pivot sequence (see Pivots above)
 *   res        one gj_result (resid is NaN)
 *   opts       NULL or options with precision GJ_PREC_FP64 and want_resid 0
 *              (else GJ_E_UNSUPPORTED); zero_tol as for gj_invert
 *   ws         workspace of gj_workspace_size(GJ_OP_SOLVE, n, &m, opts) bytes,
 *              256-byte aligned
 * Every order goes through the streaming kernels.
 * Paper: eqs. 1-2 (with D^0 = B), 13-15, Obs. 2-3.
 */
gj_status gj_solve(int32_t n, int32_t m, const double *A, int64_t lda, const double *B,
                   int64_t ldb, double *X, int64_t ldx, int32_t *ipiv, int32_t *jpiv,
                   gj_result *res, const gj_opts *opts, void *ws, size_t ws_bytes, void *stream);

/*
 * gj_workspace_size -- bytes of workspace needed.
 *   op          GJ_OP_INVERT or GJ_OP_DET: n_or_batch = n, n_host unused;
 *               GJ_OP_INVERT_BATCHED: n_or_batch = batch, n_host = HOST array of
 *               orders;
 *               GJ_OP_SOLVE: n_or_batch = n, n_host = HOST pointer to m (one int32).
 * Returns 0 for invalid arguments.
 */
size_t gj_workspace_size(int32_t op, int32_t n_or_batch, const int32_t *n_host,
                         const gj_opts *opts);

/*
 * gj_dgemm -- the FP64 matrix-core product used by the refinement and by the
 * FP64 determinant of the refined path:
 *     D = alpha * (A B) + beta * C + gamma * I       (row-major, FP64)
 * A is M x K (lda), B is K x N (ldb), C and D are M x N (ldc, ldd); C may be
 * NULL when beta == 0 and may equal D (in-place update).  gamma adds to the
 * entries with row == column.  Device pointers; asynchronous on `stream`.
 * Paper: not in the paper; the Newton-Schulz step X <- X + X (I - A X) of
 * the refined path is built from two of these products.
 */
gj_status gj_dgemm(int32_t M, int32_t N, int32_t K, double alpha, const double *A, int64_t lda,
                   const double *B, int64_t ldb, double beta, const double *C, int64_t ldc,
                   double gamma, double *D, int64_t ldd, void *stream);

/*
 * gj_sgemm -- the same product in FP32 on the matrix cores
 * (v_mfma_f32_16x16x4f32, FP32 accumulation):
 *     D = alpha * (A B) + beta * C + gamma * I       (row-major, FP32)
 * Shapes, leading dimensions, aliasing and errors as for gj_dgemm.  Paper:
 * not in the paper; the delayed updates of the FP32 elimination with
 * GJ_FLAG_BLOCKED (the panel's left factors of section 1 grouped into one
 * product) are made of these products.
 */
gj_status gj_sgemm(int32_t M, int32_t N, int32_t K, float alpha, const float *A, int64_t lda,
                   const float *B, int64_t ldb, float beta, const float *C, int64_t ldc,
                   float gamma, float *D, int64_t ldd, void *stream);

/* Text for a gj_status value or a GJ_RES_* code given as (100 + code). */
const char *gj_status_string(int32_t code);

/* Largest order handled on chip (one workgroup per matrix) for an elimination
 * precision (GJ_PREC_FP64 or GJ_PREC_FP32_REFINED). */
int32_t gj_onchip_max_n(int32_t precision);

#ifdef __cplusplus
}
#endif

#endif /* GJ_H */
