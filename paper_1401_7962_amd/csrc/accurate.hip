// accurate.hip -- the refined path's optional accurate-residual phase.
//
// Newton-Schulz with residuals R = I - A X computed in FP64 stalls once
// ||R|| reaches the rounding error of the product A X, about n u cond(A), and
// the forward error of X stays at that level.  This phase computes R with
// error-free products on the FP64 matrix cores (an Ozaki-style splitting),
// so a few more updates X <- X + X R bring the forward error of X down to
// about u:
//   * A is split per row and X as a whole into three slices, A = A1 + A2 + A3
//     and X = X1 + X2 + X3, by the extraction q = fl(fl(sigma + a) - sigma)
//     with sigma = 0.75 * 2^(e - beta + 53) (e: max |a| < 2^e over the row or
//     the matrix).  Slices 1 and 2 are multiples of 2^(e - beta) and
//     2^(e - 2 beta) with at most beta + 1 significant bits; slice 3 is the
//     exact remainder.
//   * With beta = 19 and n <= 16384, every partial sum of A_s X_t for
//     s, t <= 2 is a multiple of the product of the two units and below 2^53
//     of them, so the matrix-core product is exact in any order.
//   * R = I - A1 X1 - (every other slice pair but A3 X3): the first
//     subtraction is exact (Sterbenz on the diagonal), the remaining terms
//     are at most 2^-beta |A||X| and are added in FP64; the products with a
//     third slice round at u 2^-38 |A||X| or less; the omitted A3 X3 is below
//     2^-76 |A||X|.  |A||X| is not of the order of A X = I: the entries of
//     A X cancel, by up to n max|A| max|X| (2^28 for a 256^2 matrix of
//     condition 2^20 in the tests), so the terms of order 2^-57 |A||X| have
//     to be kept.
// Control stays on the device: an update is applied while ||R||_F at least
// halves (every time after the first), at most a fixed number of times.
#include "gj_launch.h"

namespace gj {

namespace {

__device__ __forceinline__ void extract3(double a, double sig1, double sig2, double &q1, double &q2,
                                         double &q3) {
    // -ffp-contract=off and no reassociation: each line is two IEEE additions
    q1 = (sig1 + a) - sig1;
    const double r1 = a - q1;
    q2 = (sig2 + r1) - sig2;
    q3 = r1 - q2;
}

__device__ double block_max(double v) {
    __shared__ double s[256];
    const int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) s[t] = fmax(s[t], s[t + w]);
        __syncthreads();
    }
    const double m = s[0];
    __syncthreads();
    return m;
}

// A's slices: one workgroup per row (grid-stride over rows).  S holds the
// three slices one after another, each n x n with ld n.
__global__ void __launch_bounds__(256)
slice_rows_kernel(const double *__restrict__ A, int64_t lda, int n, double *__restrict__ S, int beta,
                  const int32_t *__restrict__ run) {
    if (!*run) return;
    const int64_t nn = (int64_t)n * n;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const double *Ai = A + (int64_t)i * lda;
        double m = 0.0;
        for (int j = threadIdx.x; j < n; j += 256) m = fmax(m, fabs(Ai[j]));
        m = block_max(m);
        int e = 0;
        frexp(m, &e);                       // m < 2^e
        const double sig1 = ldexp(0.75, e - beta + 53), sig2 = ldexp(0.75, e - 2 * beta + 53);
        for (int j = threadIdx.x; j < n; j += 256) {
            double q1, q2, q3;
            extract3(Ai[j], sig1, sig2, q1, q2, q3);
            S[(int64_t)i * n + j] = q1;
            S[nn + (int64_t)i * n + j] = q2;
            S[2 * nn + (int64_t)i * n + j] = q3;
        }
    }
}

// max |X| over the matrix into ctl->xmax_bits (non-negative doubles order
// like their bit patterns)
__global__ void __launch_bounds__(256)
absmax_kernel(const double *__restrict__ X, int64_t ldx, int n, RefineCtl *ctl) {
    if (!ctl->run_acc) return;
    double m = 0.0;
    for (int i = blockIdx.x; i < n; i += gridDim.x)
        for (int j = threadIdx.x; j < n; j += 256) m = fmax(m, fabs(X[(int64_t)i * ldx + j]));
    m = block_max(m);
    if (threadIdx.x == 0)
        atomicMax(&ctl->xmax_bits, (unsigned long long)__double_as_longlong(m));
}

__global__ void __launch_bounds__(256)
slice_global_kernel(const double *__restrict__ X, int64_t ldx, int n, const RefineCtl *ctl,
                    double *__restrict__ S, int beta) {
    if (!ctl->run_acc) return;
    const double m = __longlong_as_double((long long)ctl->xmax_bits);
    int e = 0;
    frexp(m, &e);
    const double sig1 = ldexp(0.75, e - beta + 53), sig2 = ldexp(0.75, e - 2 * beta + 53);
    const int64_t nn = (int64_t)n * n;
    for (int i = blockIdx.x; i < n; i += gridDim.x)
        for (int j = threadIdx.x; j < n; j += 256) {
            double q1, q2, q3;
            extract3(X[(int64_t)i * ldx + j], sig1, sig2, q1, q2, q3);
            S[(int64_t)i * n + j] = q1;
            S[nn + (int64_t)i * n + j] = q2;
            S[2 * nn + (int64_t)i * n + j] = q3;
        }
}

__global__ void acc_prepare_kernel(RefineCtl *ctl, int enabled) {
    if (threadIdx.x != 0) return;
    ctl->run_acc = (enabled && !ctl->run_fallback) ? 1 : 0;
    ctl->acc_updates = 0;
    ctl->r_acc = __builtin_inf();
    ctl->xmax_bits = 0ull;
}

// after the accurate residual of the current iterate: apply the update only
// while ||R||_F at least halves; a non-finite or zero residual stops
__global__ void __launch_bounds__(256)
acc_check_kernel(RefineCtl *ctl, int j) {
    if (!ctl->run_acc) return;
    double acc = 0.0;
    __shared__ double s[256];
    for (int i = threadIdx.x; i < ctl->nparts; i += 256) acc += ctl->partials[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double rn = sqrt(s[0]);
    const bool go = (rn <= 1.7976931348623157e308) && rn > 0.0 && (j == 0 || rn < 0.5 * ctl->r_acc);
    ctl->r_acc = (rn <= 1.7976931348623157e308) ? rn : ctl->r_acc;
    ctl->xmax_bits = 0ull;   // for the next iterate's maximum
    if (go) ctl->acc_updates += 1;
    else ctl->run_acc = 0;
}

__global__ void __launch_bounds__(256)
acc_copy_kernel(const double *__restrict__ src, int n, double *__restrict__ X, int64_t ldx,
                const RefineCtl *ctl) {
    if (!ctl->run_acc) return;
    for (int i = blockIdx.x; i < n; i += gridDim.x)
        for (int j = threadIdx.x; j < n; j += 256) X[(int64_t)i * ldx + j] = src[(int64_t)i * n + j];
}

__global__ void acc_finish_kernel(RefineCtl *ctl) {
    if (threadIdx.x != 0) return;
    ctl->run_acc = 0;
    ctl->updates += ctl->acc_updates;
}

int rows_grid(int n) { return n < 2048 ? n : 2048; }

}  // namespace

const int32_t *ctl_run_acc(const void *c) { return &((const RefineCtl *)c)->run_acc; }

hipError_t launch_acc_prepare(void *ctl, int enabled, hipStream_t s) {
    hipLaunchKernelGGL(acc_prepare_kernel, dim3(1), dim3(64), 0, s, (RefineCtl *)ctl, enabled);
    return hipGetLastError();
}

hipError_t launch_slice_rows(const double *A, int64_t lda, int n, double *S, int beta,
                             const int32_t *run, hipStream_t s) {
    hipLaunchKernelGGL(slice_rows_kernel, dim3(rows_grid(n)), dim3(256), 0, s, A, lda, n, S, beta, run);
    return hipGetLastError();
}

hipError_t launch_slice_global(const double *X, int64_t ldx, int n, void *ctl, double *S, int beta,
                               hipStream_t s) {
    hipLaunchKernelGGL(absmax_kernel, dim3(rows_grid(n)), dim3(256), 0, s, X, ldx, n, (RefineCtl *)ctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(slice_global_kernel, dim3(rows_grid(n)), dim3(256), 0, s, X, ldx, n,
                       (const RefineCtl *)ctl, S, beta);
    return hipGetLastError();
}

hipError_t launch_acc_check(void *ctl, int j, hipStream_t s) {
    hipLaunchKernelGGL(acc_check_kernel, dim3(1), dim3(256), 0, s, (RefineCtl *)ctl, j);
    return hipGetLastError();
}

hipError_t launch_acc_copy(const double *src, int n, double *X, int64_t ldx, const void *ctl,
                           hipStream_t s) {
    hipLaunchKernelGGL(acc_copy_kernel, dim3(rows_grid(n)), dim3(256), 0, s, src, n, X, ldx,
                       (const RefineCtl *)ctl);
    return hipGetLastError();
}

hipError_t launch_acc_finish(void *ctl, hipStream_t s) {
    hipLaunchKernelGGL(acc_finish_kernel, dim3(1), dim3(64), 0, s, (RefineCtl *)ctl);
    return hipGetLastError();
}

}  // namespace gj
