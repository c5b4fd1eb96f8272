// refine.hip -- the FP32-elimination + FP64-refinement path.
//
// 1. The full-pivot elimination runs in FP32 (same kernels, T = float, zero
//    threshold 0): X0, the pivot sequence, and half the HBM traffic.
// 2. Newton-Schulz in FP64 on the matrix cores:
//        R_k = I - A X_k,   X_{k+1} = X_k + X_k R_k   (so R_{k+1} = R_k^2),
//    with the guard: an update is kept only if ||R||_F decreases, and once
//    ||R||_F < 1 the loop ends at the first update that fails to halve it
//    (the FP64 rounding floor), or after max_refine_iters updates.  A result whose final ||R||_F exceeds
//    1e-2 is replaced by the plain FP64 elimination (GJ_RES_REFINE_FALLBACK).
// 3. The FP64 determinant, which FP32 pivots cannot give: A is permuted with
//    the FP32 run's row and column order, and block Gaussian elimination in
//    FP64 runs over diagonal blocks of at most 128: each diagonal block of the
//    current Schur complement is inverted (with its determinant, eq. 13) by the
//    on-chip FP64 kernel, and the trailing matrix is updated with two MFMA
//    GEMMs, S22 <- S22 - S21 (S11^-1 S12).  det A = sign(P) sign(Q) prod det S11.
// All control decisions are taken on the device (flags in RefineCtl), so the
// launch sequence is fixed and needs no host synchronisation.
#include "gj_launch.h"

namespace gj {

struct RefineCtl {
    int32_t run_ns;        // refinement still running
    int32_t run_fallback;  // plain FP64 elimination needed
    int32_t run_det;       // FP64 block determinant needed
    int32_t updates;       // Newton-Schulz updates kept
    int32_t final_buf;     // 0: iterate in X, 1: iterate in the workspace copy
    int32_t copy_back;     // 1: copy the workspace iterate into X
    int32_t always;        // constant 1 (a run flag that is always set)
    int32_t pad;
    double r;              // ||R||_F of the kept iterate
    double r0;             // ||R_0||_F
};

namespace {

__device__ double block_sum_fixed(const double *p, int np) {
    // deterministic: thread t sums a fixed strided subset, then a fixed tree
    __shared__ double s[256];
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int i = t; i < np; i += 256) acc += p[i];
    s[t] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) s[t] += s[t + w];
        __syncthreads();
    }
    return s[0];
}

__global__ void refine_start_kernel(const gj_result *res32, RefineCtl *ctl) {
    if (threadIdx.x != 0) return;
    const bool ok = res32->code == GJ_RES_OK;
    ctl->run_ns = ok ? 1 : 0;
    ctl->run_fallback = ok ? 0 : 1;
    ctl->run_det = 0;
    ctl->updates = 0;
    ctl->final_buf = 0;
    ctl->copy_back = 0;
    ctl->always = 1;
    ctl->r = __builtin_inf();
    ctl->r0 = __builtin_inf();
}

__global__ void __launch_bounds__(256)
refine_resid0_kernel(const double *partials, int np, RefineCtl *ctl) {
    if (!ctl->run_ns) return;
    const double r = sqrt(block_sum_fixed(partials, np));
    if (threadIdx.x == 0) {
        ctl->r0 = r;
        ctl->r = r;
        if (!(r <= 1.7976931348623157e308)) ctl->run_ns = 0;   // non-finite: finish decides
        else if (r == 0.0) ctl->run_ns = 0;                      // already exact
    }
}

__global__ void __launch_bounds__(256)
refine_after_update_kernel(const double *partials, int np, RefineCtl *ctl, int it, int max_iters,
                           double stall) {
    if (!ctl->run_ns) return;
    const double rn = sqrt(block_sum_fixed(partials, np));
    if (threadIdx.x != 0) return;
    const double r = ctl->r;
    if (!(rn < r)) {                     // no progress (or NaN): keep the previous iterate
        ctl->final_buf = (it - 1) & 1;
        ctl->run_ns = 0;
        return;
    }
    ctl->r = rn;
    ctl->updates = it;
    ctl->final_buf = it & 1;
    // the halving test means "rounding floor reached" only in the contraction
    // regime ||R|| < 1, where ||R_{k+1}|| <= ||R_k||^2
    if ((r < 1.0 && rn > stall * r) || it >= max_iters || rn == 0.0) ctl->run_ns = 0;
}

__global__ void refine_finish_kernel(RefineCtl *ctl, double accept, int det_wanted) {
    if (threadIdx.x != 0) return;
    ctl->run_ns = 0;
    if (!ctl->run_fallback) {
        if (!(ctl->r <= accept)) ctl->run_fallback = 1;
    }
    ctl->copy_back = (!ctl->run_fallback && ctl->final_buf == 1) ? 1 : 0;
    ctl->run_det = (!ctl->run_fallback && det_wanted) ? 1 : 0;
}

__global__ void __launch_bounds__(256)
copy_flagged_kernel(const double *src, int64_t lds, double *dst, int64_t ldd, int n,
                    const int32_t *flag) {
    if (!*flag) return;
    for (int i = blockIdx.x; i < n; i += gridDim.x)
        for (int j = threadIdx.x; j < n; j += 256) dst[(int64_t)i * ldd + j] = src[(int64_t)i * lds + j];
}

// After the fallback run: mark its outcome.
__global__ void refine_fallback_mark_kernel(gj_result *res, const RefineCtl *ctl) {
    if (threadIdx.x != 0 || !ctl->run_fallback) return;
    if (res->code == GJ_RES_OK) res->code = GJ_RES_REFINE_FALLBACK;
    res->refine_iters = ctl->updates;
}

// Row / column order of the FP32 run as permutations: the pivoted matrix is
// B(a, b) = A(rows[a], cols[b]).  The swaps are replayed in step order.
__global__ void perms_from_pivots_kernel(const int32_t *ipiv, const int32_t *jpiv, int n,
                                         int32_t *rows, int32_t *cols, const int32_t *flag) {
    if (!*flag || threadIdx.x != 0) return;
    for (int i = 0; i < n; ++i) { rows[i] = i; cols[i] = i; }
    for (int k = 0; k < n; ++k) {
        const int r = ipiv[k], c = jpiv[k];
        int t = rows[k]; rows[k] = rows[r]; rows[r] = t;
        t = cols[k]; cols[k] = cols[c]; cols[c] = t;
    }
}

__global__ void __launch_bounds__(256)
gather_perm_kernel(const double *A, int64_t lda, const int32_t *rows, const int32_t *cols, int n,
                   double *B, int64_t ldb, const int32_t *flag) {
    if (!*flag) return;
    for (int a = blockIdx.x; a < n; a += gridDim.x) {
        const double *Ar = A + (int64_t)rows[a] * lda;
        for (int b = threadIdx.x; b < n; b += 256) B[(int64_t)a * ldb + b] = Ar[cols[b]];
    }
}

// det A = sign(P) sign(Q) prod det(S11) over the diagonal blocks.
__global__ void det_combine_kernel(const gj_result *blocks, int nblocks, const int32_t *ipiv,
                                   const int32_t *jpiv, int n, gj_result *res, RefineCtl *ctl) {
    if (!ctl->run_det || threadIdx.x != 0) return;
    int sign = 1;
    for (int k = 0; k < n; ++k) {
        if (ipiv[k] != k) sign = -sign;
        if (jpiv[k] != k) sign = -sign;
    }
    DetAcc<double> d;
    d.init();
    bool bad = false;
    for (int b = 0; b < nblocks; ++b) {
        const gj_result br = blocks[b];
        if (br.code != GJ_RES_OK) { bad = true; break; }
        d.mul(br.det_mant);      // exact power-of-two rescaling: mantissa product only
        d.e += br.det_exp;
        sign *= br.det_sign;
    }
    res->refine_iters = ctl->updates;
    if (bad) {
        res->det_sign = 0;
        res->det_mant = 0.0;
        res->det_exp = 0;
        res->det = 0.0;
        res->logabsdet = -__builtin_inf();
        return;
    }
    res->det_sign = sign;
    res->det_mant = d.m;
    res->det_exp = d.e;
    res->det = ldexp64((double)sign * d.m, d.e);
    res->logabsdet = log(d.m) + (double)d.e * 0.69314718055994530942;
}

__global__ void refine_iters_kernel(gj_result *res, const RefineCtl *ctl) {
    if (threadIdx.x == 0 && !ctl->run_fallback) res->refine_iters = ctl->updates;
}

// Per-workgroup sums of squares of an n x n matrix (for ||.||_F).
__global__ void __launch_bounds__(256)
sumsq_kernel(const double *M, int64_t ld, int n, double *partials) {
    double acc = 0.0;
    for (int i = blockIdx.x; i < n; i += gridDim.x)
        for (int j = threadIdx.x; j < n; j += 256) {
            const double v = M[(int64_t)i * ld + j];
            acc = fma(v, v, acc);
        }
    __shared__ double s[256];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
}

// resid = ||R||_F / (||A||_F ||X||_F) from three partial-sum arrays.
__global__ void __launch_bounds__(256)
resid_kernel(const double *pr, int nr, const double *pa, int na, const double *px, int nx,
             gj_result *res) {
    const double r = block_sum_fixed(pr, nr);
    const double a = block_sum_fixed(pa, na);
    const double x = block_sum_fixed(px, nx);
    if (threadIdx.x == 0) res->resid = sqrt(r) / (sqrt(a) * sqrt(x));
}

}  // namespace

size_t refine_ctl_bytes() { return sizeof(RefineCtl); }
const int32_t *ctl_run_ns(const void *c) { return &((const RefineCtl *)c)->run_ns; }
const int32_t *ctl_run_fallback(const void *c) { return &((const RefineCtl *)c)->run_fallback; }
const int32_t *ctl_run_det(const void *c) { return &((const RefineCtl *)c)->run_det; }
const int32_t *ctl_copy_back(const void *c) { return &((const RefineCtl *)c)->copy_back; }
const int32_t *ctl_always(const void *c) { return &((const RefineCtl *)c)->always; }

#define GJ_CHECK_LAUNCH() do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

hipError_t launch_refine_start(const gj_result *res32, void *ctl, hipStream_t s) {
    hipLaunchKernelGGL(refine_start_kernel, dim3(1), dim3(64), 0, s, res32, (RefineCtl *)ctl);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_refine_resid0(const double *partials, int np, void *ctl, hipStream_t s) {
    hipLaunchKernelGGL(refine_resid0_kernel, dim3(1), dim3(256), 0, s, partials, np, (RefineCtl *)ctl);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_refine_after_update(const double *partials, int np, void *ctl, int it,
                                      int max_iters, double stall, hipStream_t s) {
    hipLaunchKernelGGL(refine_after_update_kernel, dim3(1), dim3(256), 0, s, partials, np,
                       (RefineCtl *)ctl, it, max_iters, stall);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_refine_finish(void *ctl, double accept, int det_wanted, hipStream_t s) {
    hipLaunchKernelGGL(refine_finish_kernel, dim3(1), dim3(64), 0, s, (RefineCtl *)ctl, accept,
                       det_wanted);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_copy_flagged(const double *src, int64_t lds, double *dst, int64_t ldd, int n,
                               const int32_t *flag, hipStream_t s) {
    const int grid = n < 1024 ? n : 1024;
    hipLaunchKernelGGL(copy_flagged_kernel, dim3(grid), dim3(256), 0, s, src, lds, dst, ldd, n, flag);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_fallback_mark(gj_result *res, const void *ctl, hipStream_t s) {
    hipLaunchKernelGGL(refine_fallback_mark_kernel, dim3(1), dim3(64), 0, s, res,
                       (const RefineCtl *)ctl);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_perms_from_pivots(const int32_t *ipiv, const int32_t *jpiv, int n, int32_t *rows,
                                    int32_t *cols, const int32_t *flag, hipStream_t s) {
    hipLaunchKernelGGL(perms_from_pivots_kernel, dim3(1), dim3(64), 0, s, ipiv, jpiv, n, rows, cols, flag);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_gather_perm(const double *A, int64_t lda, const int32_t *rows, const int32_t *cols,
                              int n, double *B, int64_t ldb, const int32_t *flag, hipStream_t s) {
    const int grid = n < 2048 ? n : 2048;
    hipLaunchKernelGGL(gather_perm_kernel, dim3(grid), dim3(256), 0, s, A, lda, rows, cols, n, B, ldb, flag);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_det_combine(const gj_result *blocks, int nblocks, const int32_t *ipiv,
                              const int32_t *jpiv, int n, gj_result *res, void *ctl, hipStream_t s) {
    hipLaunchKernelGGL(det_combine_kernel, dim3(1), dim3(64), 0, s, blocks, nblocks, ipiv, jpiv, n,
                       res, (RefineCtl *)ctl);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_refine_iters(gj_result *res, const void *ctl, hipStream_t s) {
    hipLaunchKernelGGL(refine_iters_kernel, dim3(1), dim3(64), 0, s, res, (const RefineCtl *)ctl);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
int sumsq_blocks(int n) { return n < 1024 ? n : 1024; }
hipError_t launch_sumsq(const double *M, int64_t ld, int n, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(sumsq_kernel, dim3(sumsq_blocks(n)), dim3(256), 0, s, M, ld, n, partials);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_resid(const double *pr, int nr, const double *pa, int na, const double *px, int nx,
                        gj_result *res, hipStream_t s) {
    hipLaunchKernelGGL(resid_kernel, dim3(1), dim3(256), 0, s, pr, nr, pa, na, px, nx, res);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}

}  // namespace gj
