/* Exercises every entry point of oracle/gj_oracle.c on small inputs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer: random,
 * singular, tied and non-finite matrices, every pivot rule, the first-steps
 * and OpenMP forms, the batched wrapper, the solve and the static-pivot LU.
 * Exit status 0 when every call returned; a sanitizer report aborts. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t code, rank, det_sign, refine_iters;
    double det_mant;
    int64_t det_exp;
    double det, logabsdet, resid;
} ora_result;

int ora_gj_invert_f64(int, const double *, int64_t, double, double *, int32_t *, int32_t *, ora_result *);
int ora_gj_invert_f64_rule(int, const double *, int64_t, double, int, double *, int32_t *, int32_t *, ora_result *);
int ora_gj_invert_f64_first_steps(int, const double *, int64_t, double, double *, int32_t *, int32_t *,
                                  ora_result *, int, double *);
int ora_gj_invert_f32(int, const float *, int64_t, double, float *, int32_t *, int32_t *, ora_result *);
int ora_gj_invert_f80(int, const double *, int64_t, double, double *, int32_t *, int32_t *, ora_result *);
int ora_gj_invert_f64_par(int, const double *, int64_t, double, double *, int32_t *, int32_t *, ora_result *,
                          int, int);
int ora_gj_invert_f80_par(int, const double *, int64_t, double, double *, int32_t *, int32_t *, ora_result *, int);
int ora_gj_invert_batched(int, const int32_t *, const int64_t *, const double *, double *, const int64_t *,
                          int32_t *, int32_t *, ora_result *, double, int, int);
int ora_gj_solve_f64(int, int, const double *, int64_t, const double *, int64_t, double, double *, int64_t,
                     int32_t *, int32_t *, ora_result *);
int ora_gj_augmented_f64(int, const double *, int64_t, double, double *, int32_t *, int32_t *, ora_result *);
int ora_lu_static_det_f64(int, const double *, int64_t, const int32_t *, const int32_t *, ora_result *);

static uint64_t state = 88172645463325252ull;
static double rnd(void) {   /* xorshift64, uniform in [-1, 1) */
    state ^= state << 13; state ^= state >> 7; state ^= state << 17;
    return (double)(state >> 11) * 0x1p-52 - 1.0;
}

int main(void) {
    const int sizes[] = {1, 2, 3, 7, 16, 33};
    for (unsigned s = 0; s < sizeof(sizes) / sizeof(sizes[0]); ++s) {
        const int n = sizes[s];
        double *A = malloc(sizeof(double) * n * n), *X = malloc(sizeof(double) * n * n);
        float *Af = malloc(sizeof(float) * n * n), *Xf = malloc(sizeof(float) * n * n);
        double *B = malloc(sizeof(double) * n * 3), *Y = malloc(sizeof(double) * n * 3);
        double *piv = malloc(sizeof(double) * n);
        int32_t *ip = malloc(sizeof(int32_t) * n), *jp = malloc(sizeof(int32_t) * n);
        ora_result r;
        for (int variant = 0; variant < 4; ++variant) {
            for (int i = 0; i < n * n; ++i) A[i] = rnd();
            if (variant == 1 && n >= 3)                       /* exactly singular */
                for (int i = 0; i < n; ++i) A[i * n + n - 1] = A[i * n] + A[i * n + 1];
            if (variant == 2) A[(n * n) / 2] = NAN;           /* non-finite */
            if (variant == 3)                                 /* ties everywhere */
                for (int i = 0; i < n * n; ++i) A[i] = (i % 3) ? 1.0 : -1.0;
            for (int i = 0; i < n * n; ++i) Af[i] = (float)A[i];
            for (int i = 0; i < n * 3; ++i) B[i] = rnd();
            ora_gj_invert_f64(n, A, n, -1.0, X, ip, jp, &r);
            for (int rule = 0; rule < 3; ++rule) ora_gj_invert_f64_rule(n, A, n, -1.0, rule, X, ip, jp, &r);
            ora_gj_invert_f64_first_steps(n, A, n, -1.0, X, ip, jp, &r, n / 2, piv);
            ora_gj_invert_f32(n, Af, n, 0.0, Xf, ip, jp, &r);
            ora_gj_invert_f80(n, A, n, -1.0, X, ip, jp, &r);
            ora_gj_invert_f64_par(n, A, n, -1.0, X, ip, jp, &r, 3, n);
            ora_gj_invert_f80_par(n, A, n, -1.0, X, ip, jp, &r, 2);
            ora_gj_solve_f64(n, 3, A, n, B, 3, -1.0, Y, 3, ip, jp, &r);
            ora_gj_augmented_f64(n, A, n, -1.0, X, ip, jp, &r);
            ora_gj_invert_f64(n, A, n, -1.0, X, ip, jp, &r);
            if (r.code == 0) ora_lu_static_det_f64(n, A, n, ip, jp, &r);
        }
        free(A); free(X); free(Af); free(Xf); free(B); free(Y); free(piv); free(ip); free(jp);
    }
    /* batched: orders 1..20 packed back to back, FP64 and FP32 models */
    int32_t nn[20]; int64_t off[20], poff[20]; int64_t tot = 0, tp = 0;
    for (int b = 0; b < 20; ++b) { nn[b] = b + 1; off[b] = tot; poff[b] = tp; tot += (int64_t)nn[b] * nn[b]; tp += nn[b]; }
    double *A = malloc(sizeof(double) * tot), *X = malloc(sizeof(double) * tot);
    int32_t *ip = malloc(sizeof(int32_t) * tp), *jp = malloc(sizeof(int32_t) * tp);
    ora_result res[20];
    for (int64_t i = 0; i < tot; ++i) A[i] = rnd();
    for (int prec = 0; prec < 2; ++prec)
        if (ora_gj_invert_batched(20, nn, off, A, X, poff, ip, jp, res, -1.0, prec, 4) != 0) return 1;
    free(A); free(X); free(ip); free(jp);
    printf("oracle driver: done\n");
    return 0;
}
