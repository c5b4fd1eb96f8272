/*
 * gj_oracle.c -- plain, slow, obviously correct CPU oracle for full-pivot
 * Gauss-Jordan inversion (Anghel Drugarin, "Numerical application and Turbo C
 * program using the Gauss-Jordan method", arXiv:1401.7962).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which
 * only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load.  It shares no code, header or constant with the HIP
 * library; the two meet only through seeded inputs.
 *
 * What is computed (paper section 2):
 *   - initialisation A^0 = A, D^0 = I                         (eqs. 1-2)
 *   - at step k: pivot search by maximum |a| over the trailing block, with a
 *     swap of rows k,i and columns k,j                         (Obs. 2 and 3)
 *   - the pivot row of A and D divided by the pivot            (eq. 14)
 *   - every other row i gets -a_ik times the new pivot row     (eq. 15 and the
 *     prose that follows it: the D update uses the D pivot row)
 *   - at the end A^n = I, A^-1 = D^n                           (eqs. 11-12)
 *   - det A = product of the pivots                            (eq. 13)
 *   - the row and column swaps are undone in reverse order     (Obs. 3 and the
 *     conclusions)
 *   - a pivot that is null or below a preset zero threshold, when no other
 *     candidate is usable, means A is singular                 (Obs. 2)
 *
 * Readings of points the paper leaves open:
 *   - the D half is stored in place in the columns that A no longer needs, so
 *     one n x n array holds [A|D] (the work-skipping form, eqs. 3-10);
 *   - eq. 14 uses correctly rounded division; the pivot slot becomes 1/p;
 *   - eq. 15 is one fused multiply-add per element: w = fma(-q, w_kj, w);
 *   - ties between equal |a| go to the lowest row, then the lowest column, of
 *     the current (already swapped) matrix = first maximum in row-major order;
 *   - the determinant sign is (-1)^(number of non-trivial row and column
 *     swaps); the product is kept as mantissa in [0.5,1) times 2^e;
 *   - default zero threshold tau = n * 2^-52 * (largest |a| of A); a step is
 *     singular if its pivot candidate m satisfies m == 0 or m < tau;
 *   - any NaN or infinity among the candidates stops the run (NONFINITE).
 *
 * The routine is written once as a macro and instantiated for double (the
 * FP64 oracle), long double (x87 64-bit mantissa: the "truth" used for
 * forward errors) and float (a CPU model of an FP32 elimination).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -fPIC -shared
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Result record, laid out field by field like the library's public record so
 * that the same ctypes structure reads both.  Codes: 0 ok, 1 singular,
 * 2 non-finite, 3 refinement fell back. */
typedef struct {
    int32_t code, rank, det_sign, refine_iters;
    double det_mant;
    int64_t det_exp;
    double det, logabsdet, resid;
} ora_result;

enum { ORA_OK = 0, ORA_SINGULAR = 1, ORA_NONFINITE = 2, ORA_REFINE_FALLBACK = 3 };

static double ora_ldexp64(double m, int64_t e)
{
    /* ldexp with a 64-bit exponent: saturate far outside the double range */
    if (e > 4000) e = 4000;
    if (e < -4000) e = -4000;
    return ldexp(m, (int)e);
}

static void ora_fill_failure(ora_result *res, int code, int rank, int n,
                             int32_t *ipiv, int32_t *jpiv)
{
    res->code = code;
    res->rank = rank;
    res->det_sign = 0;
    res->det_mant = 0.0;
    res->det_exp = 0;
    if (code == ORA_SINGULAR) {
        res->det = 0.0;
        res->logabsdet = -INFINITY;
    } else {
        res->det = NAN;
        res->logabsdet = NAN;
    }
    for (int k = rank; k < n; ++k) {
        if (ipiv) ipiv[k] = -1;
        if (jpiv) jpiv[k] = -1;
    }
}

/*
 * Pivot rules.  0: the text's rule (Obs. 2-3): largest |a| over the trailing
 * block, ties to the first in row-major order, row and column swaps.
 * 1: partial pivoting on |a|: largest |a| in column k, rows k..n-1, first
 * wins; row swaps only.  2: the rule of the program in section 3: the row
 * with the largest positive value in column k (strictly greater, starting
 * from 0), else row k itself; row swaps only.  Rules 1 and 2 have no preset
 * threshold (the program has none): with zero_tol < 0 only an exactly zero
 * pivot is singular.
 *
 * GJ_INPLACE(NAME, T, FABS, FMA, FREXP, ISFIN)
 *
 * int NAME(int n, const T *A, int64_t lda, double zero_tol,
 *          T *X, int32_t *ipiv, int32_t *jpiv, ora_result *res)
 *
 * A: n x n row-major, leading dimension lda.  X: n x n row-major, ld n,
 * receives A^-1 (all NaN when the run stops early).  ipiv[k] / jpiv[k]: the
 * row / column (0-based, of the current matrix) swapped with k at step k,
 * -1 for steps not taken.  zero_tol < 0 selects the default threshold.
 * Returns res->code.
 */
#define GJ_INPLACE(NAME, T, FABS, FMA, FREXP, ISFIN, EPS_DEFAULT)                  \
static int NAME##_run(int n, const T *A, int64_t lda, double zero_tol, T *X,       \
                      int32_t *ipiv, int32_t *jpiv, ora_result *res,               \
                      int max_steps, double *pivots, int rule);                    \
int NAME(int n, const T *A, int64_t lda, double zero_tol, T *X,                    \
         int32_t *ipiv, int32_t *jpiv, ora_result *res)                            \
{                                                                                  \
    return NAME##_run(n, A, lda, zero_tol, X, ipiv, jpiv, res, n, NULL, 0);        \
}                                                                                  \
/* another pivot rule (see the rule codes above the macro)                  */   \
int NAME##_rule(int n, const T *A, int64_t lda, double zero_tol, int rule, T *X,   \
                int32_t *ipiv, int32_t *jpiv, ora_result *res)                     \
{                                                                                  \
    return NAME##_run(n, A, lda, zero_tol, X, ipiv, jpiv, res, n, NULL, rule);     \
}                                                                                  \
/* the first max_steps steps only, recording each pivot value; the working  */   \
/* array is left as it stands after those steps (no depivoting)             */   \
int NAME##_first_steps(int n, const T *A, int64_t lda, double zero_tol, T *X,      \
                       int32_t *ipiv, int32_t *jpiv, ora_result *res,              \
                       int max_steps, double *pivots)                              \
{                                                                                  \
    return NAME##_run(n, A, lda, zero_tol, X, ipiv, jpiv, res, max_steps, pivots, 0); \
}                                                                                  \
static int NAME##_run(int n, const T *A, int64_t lda, double zero_tol, T *X,       \
                      int32_t *ipiv, int32_t *jpiv, ora_result *res,               \
                      int max_steps, double *pivots, int rule)                     \
{                                                                                  \
    T *W = X;                                   /* in-place working array */       \
    for (int i = 0; i < n; ++i)                                                    \
        for (int j = 0; j < n; ++j)                                                \
            W[(int64_t)i * n + j] = A[(int64_t)i * lda + j];   /* eqs. 1-2 */      \
    int sign = 1;                                                                  \
    T m_acc = (T)1;                                                                \
    int64_t e_acc = 0;                                                             \
    T tau = (T)zero_tol;                                                           \
    res->refine_iters = 0;                                                         \
    res->resid = NAN;                                                              \
    for (int k = 0; k < n; ++k) {                                                  \
        if (k == max_steps) return ORA_OK;                                         \
        /* pivot search over the trailing block, first maximum in row-major   */  \
        /* order (Obs. 2 and 3)                                               */  \
        T best = (T)-1;                                                            \
        int r = -1, c = -1, nonfinite = 0;                                         \
        if (rule == 0) {                                                           \
        for (int i = k; i < n; ++i)                                                \
            for (int j = k; j < n; ++j) {                                          \
                T v = FABS(W[(int64_t)i * n + j]);                                 \
                if (!ISFIN(v)) nonfinite = 1;                                      \
                if (v > best) { best = v; r = i; c = j; }                          \
            }                                                                      \
        } else {   /* column k only, rows k..n-1; no column swap            */    \
            T q = (T)0;                                                            \
            c = k;                                                                 \
            r = (rule == 2) ? k : -1;                                              \
            for (int i = k; i < n; ++i) {                                          \
                T v = W[(int64_t)i * n + k];                                       \
                if (!ISFIN(v)) nonfinite = 1;                                      \
                if (rule == 1) {                /* largest |a|, first wins   */    \
                    if (FABS(v) > best) { best = FABS(v); r = i; }                 \
                } else if (v > q) {             /* largest positive value    */    \
                    q = v; r = i;                                                  \
                }                                                                  \
            }                                                                      \
            if (rule == 2) best = FABS(W[(int64_t)r * n + k]);                     \
        }                                                                          \
        if (nonfinite) {                                                           \
            ora_fill_failure(res, ORA_NONFINITE, k, n, ipiv, jpiv);                \
            for (int64_t t = 0; t < (int64_t)n * n; ++t) W[t] = (T)NAN;            \
            return ORA_NONFINITE;                                                  \
        }                                                                          \
        if (k == 0 && zero_tol < 0)   /* preset zero threshold (none: 0) */         \
            tau = (rule == 0) ? (T)n * (T)(EPS_DEFAULT) * best : (T)0;             \
        if (best == (T)0 || best < tau) {           /* Obs. 2: singular */         \
            ora_fill_failure(res, ORA_SINGULAR, k, n, ipiv, jpiv);                 \
            for (int64_t t = 0; t < (int64_t)n * n; ++t) W[t] = (T)NAN;            \
            return ORA_SINGULAR;                                                   \
        }                                                                          \
        ipiv[k] = r;                                                               \
        jpiv[k] = c;                                                               \
        if (r != k) {                               /* swap rows k and r */        \
            for (int j = 0; j < n; ++j) {                                          \
                T t = W[(int64_t)k * n + j];                                       \
                W[(int64_t)k * n + j] = W[(int64_t)r * n + j];                     \
                W[(int64_t)r * n + j] = t;                                         \
            }                                                                      \
            sign = -sign;                                                          \
        }                                                                          \
        if (c != k) {                               /* swap columns k and c */     \
            for (int i = 0; i < n; ++i) {                                          \
                T t = W[(int64_t)i * n + k];                                       \
                W[(int64_t)i * n + k] = W[(int64_t)i * n + c];                     \
                W[(int64_t)i * n + c] = t;                                         \
            }                                                                      \
            sign = -sign;                                                          \
        }                                                                          \
        T p = W[(int64_t)k * n + k];                /* the pivot */                \
        if (pivots) pivots[k] = (double)p;                                         \
        {   /* eq. 13: running product of pivots as mantissa * 2^e */              \
            int e1, e2;                                                            \
            T f = FREXP(p, &e1);                                                   \
            m_acc = m_acc * f;                                                     \
            e_acc += e1;                                                           \
            m_acc = FREXP(m_acc, &e2);                                             \
            e_acc += e2;                                                           \
        }                                                                          \
        /* eq. 14: pivot row divided by the pivot; slot (k,k) becomes 1/p */       \
        W[(int64_t)k * n + k] = (T)1;                                              \
        for (int j = 0; j < n; ++j)                                                \
            W[(int64_t)k * n + j] = W[(int64_t)k * n + j] / p;                     \
        /* eq. 15: every other row minus a_ik times the new pivot row */           \
        for (int i = 0; i < n; ++i) {                                              \
            if (i == k) continue;                                                  \
            T q = W[(int64_t)i * n + k];                                           \
            W[(int64_t)i * n + k] = (T)0;                                          \
            for (int j = 0; j < n; ++j)                                            \
                W[(int64_t)i * n + j] = FMA(-q, W[(int64_t)k * n + j],             \
                                            W[(int64_t)i * n + j]);                \
        }                                                                          \
    }                                                                              \
    /* undo the swaps in reverse order: row swaps of A come back as column     */  \
    /* swaps of the result and column swaps of A as row swaps                  */  \
    for (int k = n - 1; k >= 0; --k) {                                             \
        int r = ipiv[k], c = jpiv[k];                                              \
        if (r != k)                                                                \
            for (int i = 0; i < n; ++i) {                                          \
                T t = W[(int64_t)i * n + k];                                       \
                W[(int64_t)i * n + k] = W[(int64_t)i * n + r];                     \
                W[(int64_t)i * n + r] = t;                                         \
            }                                                                      \
        if (c != k)                                                                \
            for (int j = 0; j < n; ++j) {                                          \
                T t = W[(int64_t)k * n + j];                                       \
                W[(int64_t)k * n + j] = W[(int64_t)c * n + j];                     \
                W[(int64_t)c * n + j] = t;                                         \
            }                                                                      \
    }                                                                              \
    res->code = ORA_OK;                                                            \
    res->rank = n;                                                                 \
    res->det_sign = (m_acc < 0) ? -sign : sign;                                    \
    res->det_mant = (double)FABS(m_acc);                                           \
    res->det_exp = e_acc;                                                          \
    res->det = ora_ldexp64((double)sign * (double)m_acc, e_acc);                   \
    res->logabsdet = log(res->det_mant) + (double)e_acc * 0.69314718055994530942;  \
    return ORA_OK;                                                                 \
}

static int isfin_d(double v) { return isfinite(v); }
static int isfin_l(long double v) { return isfinite(v); }
static int isfin_f(float v) { return isfinite(v); }

GJ_INPLACE(ora_gj_invert_f64, double, fabs, fma, frexp, isfin_d, 0x1p-52)
GJ_INPLACE(ora_gj_invert_f32, float, fabsf, fmaf, frexpf, isfin_f, 0.0)

/*
 * The same elimination (full search only) with the independent work of each
 * step shared among `nthreads` OpenMP threads, so that the oracle can be timed
 * on every host core.  Nothing about the arithmetic changes:
 *   - the search splits rows k..n-1 into contiguous ranges, one per thread;
 *     each range keeps its first maximum in row-major order, and the ranges
 *     are merged in row order with the same strict '>', which gives the first
 *     maximum of the whole block -- the serial winner;
 *   - eq. 15 updates each row i != k on its own (every row reads only the
 *     pivot row, which no thread writes during the update);
 *   - swaps, the pivot, the determinant and the depivoting stay serial.
 * So X, the pivots and the determinant equal the serial function's bit for
 * bit (a test checks it).  `max_steps` < n stops after that many steps
 * without depivoting, as the _first_steps form does (used to time a sample).
 */
#define GJ_INPLACE_PAR(NAME, T, FABS, FMA, FREXP, ISFIN, EPS_DEFAULT)              \
int NAME(int n, const T *A, int64_t lda, double zero_tol, T *X, int32_t *ipiv,     \
         int32_t *jpiv, ora_result *res, int nthreads, int max_steps)              \
{                                                                                  \
    if (nthreads < 1) nthreads = 1;                                                \
    T *sb = (T *)malloc(sizeof(T) * (size_t)nthreads);                             \
    int *sr = (int *)malloc(sizeof(int) * (size_t)nthreads * 3);                   \
    if (!sb || !sr) { free(sb); free(sr); return -1; }                             \
    T *W = X;                                                                      \
    _Pragma("omp parallel for num_threads(nthreads) schedule(static)")            \
    for (int i = 0; i < n; ++i)                                                    \
        for (int j = 0; j < n; ++j)                                                \
            W[(int64_t)i * n + j] = A[(int64_t)i * lda + j];   /* eqs. 1-2 */      \
    int sign = 1;                                                                  \
    T m_acc = (T)1;                                                                \
    int64_t e_acc = 0;                                                             \
    T tau = (T)zero_tol;                                                           \
    res->refine_iters = 0;                                                         \
    res->resid = NAN;                                                              \
    for (int k = 0; k < n; ++k) {                                                  \
        if (k == max_steps) { free(sb); free(sr); return ORA_OK; }                 \
        int used = 1;                                                              \
        _Pragma("omp parallel num_threads(nthreads)")                              \
        {                                                                          \
            const int id = omp_get_thread_num(), cnt = omp_get_num_threads();     \
            const int64_t rows = n - k;                                            \
            const int lo = k + (int)(rows * id / cnt);                             \
            const int hi = k + (int)(rows * (id + 1) / cnt);                       \
            T best = (T)-1;                                                        \
            int r = -1, c = -1, nonfinite = 0;                                     \
            for (int i = lo; i < hi; ++i)                                          \
                for (int j = k; j < n; ++j) {                                      \
                    T v = FABS(W[(int64_t)i * n + j]);                             \
                    if (!ISFIN(v)) nonfinite = 1;                                  \
                    if (v > best) { best = v; r = i; c = j; }                      \
                }                                                                  \
            sb[id] = best;                                                         \
            sr[3 * id] = r; sr[3 * id + 1] = c; sr[3 * id + 2] = nonfinite;        \
            if (id == 0) used = cnt;                                               \
        }                                                                          \
        /* merge in row order: strict '>' keeps the earliest range's maximum */   \
        T best = (T)-1;                                                            \
        int r = -1, c = -1, nonfinite = 0;                                         \
        for (int id = 0; id < used; ++id) {                                        \
            nonfinite |= sr[3 * id + 2];                                           \
            if (sb[id] > best) { best = sb[id]; r = sr[3 * id]; c = sr[3 * id + 1]; } \
        }                                                                          \
        if (nonfinite) {                                                           \
            ora_fill_failure(res, ORA_NONFINITE, k, n, ipiv, jpiv);                \
            for (int64_t t = 0; t < (int64_t)n * n; ++t) W[t] = (T)NAN;            \
            free(sb); free(sr);                                                    \
            return ORA_NONFINITE;                                                  \
        }                                                                          \
        if (k == 0 && zero_tol < 0) tau = (T)n * (T)(EPS_DEFAULT) * best;          \
        if (best == (T)0 || best < tau) {                                          \
            ora_fill_failure(res, ORA_SINGULAR, k, n, ipiv, jpiv);                 \
            for (int64_t t = 0; t < (int64_t)n * n; ++t) W[t] = (T)NAN;            \
            free(sb); free(sr);                                                    \
            return ORA_SINGULAR;                                                   \
        }                                                                          \
        ipiv[k] = r;                                                               \
        jpiv[k] = c;                                                               \
        if (r != k) {                                                              \
            for (int j = 0; j < n; ++j) {                                          \
                T t = W[(int64_t)k * n + j];                                       \
                W[(int64_t)k * n + j] = W[(int64_t)r * n + j];                     \
                W[(int64_t)r * n + j] = t;                                         \
            }                                                                      \
            sign = -sign;                                                          \
        }                                                                          \
        if (c != k) {                                                              \
            for (int i = 0; i < n; ++i) {                                          \
                T t = W[(int64_t)i * n + k];                                       \
                W[(int64_t)i * n + k] = W[(int64_t)i * n + c];                     \
                W[(int64_t)i * n + c] = t;                                         \
            }                                                                      \
            sign = -sign;                                                          \
        }                                                                          \
        T p = W[(int64_t)k * n + k];                                               \
        {                                                                          \
            int e1, e2;                                                            \
            T f = FREXP(p, &e1);                                                   \
            m_acc = m_acc * f;                                                     \
            e_acc += e1;                                                           \
            m_acc = FREXP(m_acc, &e2);                                             \
            e_acc += e2;                                                           \
        }                                                                          \
        W[(int64_t)k * n + k] = (T)1;                               /* eq. 14 */  \
        for (int j = 0; j < n; ++j)                                                \
            W[(int64_t)k * n + j] = W[(int64_t)k * n + j] / p;                     \
        _Pragma("omp parallel for num_threads(nthreads) schedule(static)")        \
        for (int i = 0; i < n; ++i) {                               /* eq. 15 */  \
            if (i == k) continue;                                                  \
            T q = W[(int64_t)i * n + k];                                           \
            W[(int64_t)i * n + k] = (T)0;                                          \
            for (int j = 0; j < n; ++j)                                            \
                W[(int64_t)i * n + j] = FMA(-q, W[(int64_t)k * n + j],             \
                                            W[(int64_t)i * n + j]);                \
        }                                                                          \
    }                                                                              \
    free(sb);                                                                      \
    free(sr);                                                                      \
    for (int k = n - 1; k >= 0; --k) {                               /* Obs. 3 */  \
        int r = ipiv[k], c = jpiv[k];                                              \
        if (r != k)                                                                \
            for (int i = 0; i < n; ++i) {                                          \
                T t = W[(int64_t)i * n + k];                                       \
                W[(int64_t)i * n + k] = W[(int64_t)i * n + r];                     \
                W[(int64_t)i * n + r] = t;                                         \
            }                                                                      \
        if (c != k)                                                                \
            for (int j = 0; j < n; ++j) {                                          \
                T t = W[(int64_t)k * n + j];                                       \
                W[(int64_t)k * n + j] = W[(int64_t)c * n + j];                     \
                W[(int64_t)c * n + j] = t;                                         \
            }                                                                      \
    }                                                                              \
    res->code = ORA_OK;                                                            \
    res->rank = n;                                                                 \
    res->det_sign = (m_acc < 0) ? -sign : sign;                                    \
    res->det_mant = (double)FABS(m_acc);                                           \
    res->det_exp = e_acc;                                                          \
    res->det = ora_ldexp64((double)sign * (double)m_acc, e_acc);                   \
    res->logabsdet = log(res->det_mant) + (double)e_acc * 0.69314718055994530942;  \
    return ORA_OK;                                                                 \
}

GJ_INPLACE_PAR(ora_gj_invert_f64_par, double, fabs, fma, frexp, isfin_d, 0x1p-52)
GJ_INPLACE_PAR(ora_gj_invert_f32_par, float, fabsf, fmaf, frexpf, isfin_f, 0.0)
GJ_INPLACE_PAR(ora_gj_invert_f80_par_impl, long double, fabsl, fmal, frexpl, isfin_l, 0x1p-52)

/*
 * Many independent matrices, one serial oracle run each, shared among
 * `nthreads` OpenMP threads (dynamic schedule).  Member b: order n[b], input
 * at A + off[b] (ld n[b]), inverse at X + off[b] (ld n[b]), pivots at
 * ipiv/jpiv + piv_off[b], record res[b].  precision 0: the FP64 oracle;
 * 1: the FP32 model (input rounded to float, result widened back).
 */
int ora_gj_invert_batched(int batch, const int32_t *nn, const int64_t *off, const double *A,
                          double *X, const int64_t *piv_off, int32_t *ipiv, int32_t *jpiv,
                          ora_result *res, double zero_tol, int precision, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    int failed = 0;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1) reduction(| : failed)
    for (int b = 0; b < batch; ++b) {
        const int n = nn[b];
        if (precision == 0) {
            ora_gj_invert_f64(n, A + off[b], n, zero_tol, X + off[b], ipiv + piv_off[b],
                              jpiv + piv_off[b], &res[b]);
        } else {
            float *a = (float *)malloc(sizeof(float) * (size_t)n * n);
            float *x = (float *)malloc(sizeof(float) * (size_t)n * n);
            if (!a || !x) { failed = 1; free(a); free(x); continue; }
            for (int64_t t = 0; t < (int64_t)n * n; ++t) a[t] = (float)A[off[b] + t];
            ora_gj_invert_f32(n, a, n, zero_tol, x, ipiv + piv_off[b], jpiv + piv_off[b], &res[b]);
            for (int64_t t = 0; t < (int64_t)n * n; ++t) X[off[b] + t] = (double)x[t];
            free(a);
            free(x);
        }
    }
    return failed ? -1 : 0;
}

/* long double variant: input and output in double, arithmetic in long
 * double.  Used as the "truth" for forward errors (unit roundoff 2^-64). */
GJ_INPLACE(ora_gj_invert_f80_impl, long double, fabsl, fmal, frexpl, isfin_l, 0x1p-52)

/* the long-double run on `nthreads` threads (same results as the serial one) */
int ora_gj_invert_f80_par(int n, const double *A, int64_t lda, double zero_tol, double *X,
                          int32_t *ipiv, int32_t *jpiv, ora_result *res, int nthreads)
{
    long double *a = (long double *)malloc(sizeof(long double) * (size_t)n * n);
    long double *x = (long double *)malloc(sizeof(long double) * (size_t)n * n);
    if (!a || !x) { free(a); free(x); return -1; }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) a[(int64_t)i * n + j] = A[(int64_t)i * lda + j];
    int code = ora_gj_invert_f80_par_impl(n, a, n, zero_tol, x, ipiv, jpiv, res, nthreads, n);
    for (int64_t t = 0; t < (int64_t)n * n; ++t) X[t] = (double)x[t];
    free(a);
    free(x);
    return code;
}

int ora_gj_invert_f80(int n, const double *A, int64_t lda, double zero_tol, double *X,
                      int32_t *ipiv, int32_t *jpiv, ora_result *res)
{
    long double *a = (long double *)malloc(sizeof(long double) * (size_t)n * n);
    long double *x = (long double *)malloc(sizeof(long double) * (size_t)n * n);
    if (!a || !x) { free(a); free(x); return -1; }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) a[(int64_t)i * n + j] = A[(int64_t)i * lda + j];
    int code = ora_gj_invert_f80_impl(n, a, n, zero_tol, x, ipiv, jpiv, res);
    for (int64_t t = 0; t < (int64_t)n * n; ++t) X[t] = (double)x[t];
    free(a);
    free(x);
    return code;
}

/*
 * Literal augmented form of eqs. 1-2 and 14-15 with a general right-hand
 * side: A (n x n) and D (n x m) held in separate arrays, D^0 = B (eq. 2 has
 * D^0 = I; any B gives D^n = Q^-1 A^-1 B instead, since every row operation
 * of the elimination is applied to D as printed).  Row swaps act on both
 * halves (a left multiplication), column swaps on A only.  At the end
 * D = Q^-1 A^-1 B where Q is the product of the column swaps, so
 * A^-1 B = Q D: the column swaps come back as row swaps of D, in reverse
 * order.  X (n x m, ld ldx) receives A^-1 B, all NaN when the run stops.
 */
int ora_gj_solve_f64(int n, int m, const double *A, int64_t lda, const double *B, int64_t ldb,
                     double zero_tol, double *X, int64_t ldx, int32_t *ipiv, int32_t *jpiv,
                     ora_result *res)
{
    double *a = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *d = (double *)malloc(sizeof(double) * (size_t)n * m);
    if (!a || !d) { free(a); free(d); return -1; }
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) a[(int64_t)i * n + j] = A[(int64_t)i * lda + j];   /* eq. 1 */
        for (int j = 0; j < m; ++j) d[(int64_t)i * m + j] = B[(int64_t)i * ldb + j];   /* eq. 2, D^0 = B */
    }
    double tau = zero_tol;
    int sign = 1;
    double m_acc = 1.0;
    int64_t e_acc = 0;
    int code = ORA_OK;
    res->refine_iters = 0;
    res->resid = NAN;
    for (int k = 0; k < n; ++k) {
        double best = -1.0;
        int r = -1, c = -1, nonfinite = 0;
        for (int i = k; i < n; ++i)
            for (int j = k; j < n; ++j) {
                double v = fabs(a[(int64_t)i * n + j]);
                if (!isfinite(v)) nonfinite = 1;
                if (v > best) { best = v; r = i; c = j; }
            }
        if (nonfinite) { ora_fill_failure(res, ORA_NONFINITE, k, n, ipiv, jpiv); code = ORA_NONFINITE; break; }
        if (k == 0 && zero_tol < 0) tau = (double)n * 0x1p-52 * best;
        if (best == 0.0 || best < tau) { ora_fill_failure(res, ORA_SINGULAR, k, n, ipiv, jpiv); code = ORA_SINGULAR; break; }
        ipiv[k] = r;
        jpiv[k] = c;
        if (r != k) {
            for (int j = 0; j < n; ++j) {
                double t = a[(int64_t)k * n + j];
                a[(int64_t)k * n + j] = a[(int64_t)r * n + j];
                a[(int64_t)r * n + j] = t;
            }
            for (int j = 0; j < m; ++j) {
                double t = d[(int64_t)k * m + j];
                d[(int64_t)k * m + j] = d[(int64_t)r * m + j];
                d[(int64_t)r * m + j] = t;
            }
            sign = -sign;
        }
        if (c != k) {
            for (int i = 0; i < n; ++i) {
                double t = a[(int64_t)i * n + k];
                a[(int64_t)i * n + k] = a[(int64_t)i * n + c];
                a[(int64_t)i * n + c] = t;
            }
            sign = -sign;
        }
        double p = a[(int64_t)k * n + k];
        {
            int e1, e2;
            double f = frexp(p, &e1);
            m_acc = m_acc * f;
            e_acc += e1;
            m_acc = frexp(m_acc, &e2);
            e_acc += e2;
        }
        for (int j = 0; j < n; ++j) a[(int64_t)k * n + j] = a[(int64_t)k * n + j] / p;   /* eq. 14 */
        for (int j = 0; j < m; ++j) d[(int64_t)k * m + j] = d[(int64_t)k * m + j] / p;
        for (int i = 0; i < n; ++i) {                                                   /* eq. 15 */
            if (i == k) continue;
            double q = a[(int64_t)i * n + k];
            for (int j = 0; j < n; ++j)
                a[(int64_t)i * n + j] = fma(-q, a[(int64_t)k * n + j], a[(int64_t)i * n + j]);
            for (int j = 0; j < m; ++j)
                d[(int64_t)i * m + j] = fma(-q, d[(int64_t)k * m + j], d[(int64_t)i * m + j]);
        }
    }
    if (code == ORA_OK) {
        for (int k = n - 1; k >= 0; --k) {                                              /* A^-1 B = Q D */
            int c = jpiv[k];
            if (c != k)
                for (int j = 0; j < m; ++j) {
                    double t = d[(int64_t)k * m + j];
                    d[(int64_t)k * m + j] = d[(int64_t)c * m + j];
                    d[(int64_t)c * m + j] = t;
                }
        }
        res->code = ORA_OK;
        res->rank = n;
        res->det_sign = (m_acc < 0) ? -sign : sign;
        res->det_mant = fabs(m_acc);
        res->det_exp = e_acc;
        res->det = ora_ldexp64((double)sign * m_acc, e_acc);
        res->logabsdet = log(res->det_mant) + (double)e_acc * 0.69314718055994530942;
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < m; ++j)
            X[(int64_t)i * ldx + j] = (code == ORA_OK) ? d[(int64_t)i * m + j] : NAN;
    free(a);
    free(d);
    return code;
}

/* The augmented form with D^0 = I (eq. 2 as printed): X receives A^-1. */
int ora_gj_augmented_f64(int n, const double *A, int64_t lda, double zero_tol, double *X,
                         int32_t *ipiv, int32_t *jpiv, ora_result *res)
{
    double *eye = (double *)calloc((size_t)n * n, sizeof(double));
    if (!eye) return -1;
    for (int i = 0; i < n; ++i) eye[(int64_t)i * n + i] = 1.0;
    int code = ora_gj_solve_f64(n, n, A, lda, eye, n, zero_tol, X, n, ipiv, jpiv, res);
    free(eye);
    return code;
}

/*
 * Static-pivot FP64 LU determinant.  Applies, step by step, the row and
 * column swaps of a previous full-pivot run (ipiv, jpiv: LAPACK xGETC2
 * convention) and eliminates below the diagonal without searching:
 * l = a_ik / a_kk, a_ij <- a_ij - l * a_kj (one fma).  det = sign * prod a_kk,
 * kept as mantissa * 2^e like eq. 13's product.  A zero or non-finite pivot
 * gives code SINGULAR / NONFINITE with rank k.
 */
int ora_lu_static_det_f64(int n, const double *A, int64_t lda, const int32_t *ipiv,
                          const int32_t *jpiv, ora_result *res)
{
    double *a = (double *)malloc(sizeof(double) * (size_t)n * n);
    if (!a) return -1;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) a[(int64_t)i * n + j] = A[(int64_t)i * lda + j];
    int sign = 1;
    double m_acc = 1.0;
    int64_t e_acc = 0;
    res->refine_iters = 0;
    res->resid = NAN;
    for (int k = 0; k < n; ++k) {
        int r = ipiv[k], c = jpiv[k];
        if (r != k) {
            for (int j = 0; j < n; ++j) {
                double t = a[(int64_t)k * n + j];
                a[(int64_t)k * n + j] = a[(int64_t)r * n + j];
                a[(int64_t)r * n + j] = t;
            }
            sign = -sign;
        }
        if (c != k) {
            for (int i = 0; i < n; ++i) {
                double t = a[(int64_t)i * n + k];
                a[(int64_t)i * n + k] = a[(int64_t)i * n + c];
                a[(int64_t)i * n + c] = t;
            }
            sign = -sign;
        }
        double p = a[(int64_t)k * n + k];
        if (!isfinite(p)) {
            ora_fill_failure(res, ORA_NONFINITE, k, n, NULL, NULL);
            free(a);
            return ORA_NONFINITE;
        }
        if (p == 0.0) {
            ora_fill_failure(res, ORA_SINGULAR, k, n, NULL, NULL);
            free(a);
            return ORA_SINGULAR;
        }
        int e1, e2;
        double f = frexp(p, &e1);
        m_acc = m_acc * f;
        e_acc += e1;
        m_acc = frexp(m_acc, &e2);
        e_acc += e2;
        for (int i = k + 1; i < n; ++i) {
            double l = a[(int64_t)i * n + k] / p;
            for (int j = k + 1; j < n; ++j)
                a[(int64_t)i * n + j] = fma(-l, a[(int64_t)k * n + j], a[(int64_t)i * n + j]);
        }
    }
    free(a);
    res->code = ORA_OK;
    res->rank = n;
    res->det_sign = (m_acc < 0) ? -sign : sign;
    res->det_mant = fabs(m_acc);
    res->det_exp = e_acc;
    res->det = ora_ldexp64((double)sign * m_acc, e_acc);
    res->logabsdet = log(res->det_mant) + (double)e_acc * 0.69314718055994530942;
    return ORA_OK;
}

/* Size of the record, so the Python side can check its layout. */
int ora_result_size(void) { return (int)sizeof(ora_result); }
