// refine.hip -- the FP32-elimination + FP64-refinement path.
//
// 1. The full-pivot elimination runs in FP32 (same kernels, T = float, zero
//    threshold 0): X0, the pivot sequence, and half the HBM traffic.
// 2. Newton-Schulz in FP64 on the matrix cores:
//        R_k = I - A X_k,   X_{k+1} = X_k + X_k R_k   (so R_{k+1} = R_k^2),
//    with the guard: an update is kept only if ||R||_F decreases, and the
//    loop ends at the FP64 rounding floor, recognised as a kept update that
//    contracted neither by half nor to within twice the quadratic bound
//    ||R_{k+1}|| <= ||R_k||^2 (rn > max(r/2, 2 r^2)), or after
//    max_refine_iters updates.  A result whose final ||R||_F exceeds 1e-2 is
//    replaced by the plain FP64 elimination (GJ_RES_REFINE_FALLBACK).
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
    const double v = s[0];
    __syncthreads();
    return v;
}

__global__ void refine_bind_kernel(RefineCtl *ctl, gj_result *res, double *partials, int nparts) {
    if (threadIdx.x != 0) return;
    ctl->res = res;
    ctl->partials = partials;
    ctl->nparts = nparts;
}

__global__ void refine_start_kernel(RefineCtl *ctls, int count) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= count) return;
    RefineCtl *ctl = ctls + m;
    const bool ok = ctl->res->code == GJ_RES_OK;
    ctl->run_ns = ok ? 1 : 0;
    ctl->run_fallback = ok ? 0 : 1;
    ctl->run_det = 0;
    ctl->updates = 0;
    ctl->final_buf = 0;
    ctl->copy_back = 0;
    ctl->always = 1;
    ctl->r = __builtin_inf();
    ctl->r0 = __builtin_inf();
    ctl->run_acc = 0;
    ctl->acc_updates = 0;
    ctl->r_acc = __builtin_inf();
    ctl->xmax_bits = 0ull;
}

__global__ void __launch_bounds__(256)
refine_resid0_kernel(RefineCtl *ctls) {
    RefineCtl *ctl = ctls + blockIdx.x;
    if (!ctl->run_ns) return;
    const double r = sqrt(block_sum_fixed(ctl->partials, ctl->nparts));
    if (threadIdx.x == 0) {
        ctl->r0 = r;
        ctl->r = r;
        if (!(r <= 1.7976931348623157e308)) ctl->run_ns = 0;   // non-finite: finish decides
        else if (r == 0.0) ctl->run_ns = 0;                      // already exact
    }
}

__global__ void __launch_bounds__(256)
refine_after_update_kernel(RefineCtl *ctls, int it, int max_iters, double stall) {
    RefineCtl *ctl = ctls + blockIdx.x;
    if (!ctl->run_ns) return;
    const double rn = sqrt(block_sum_fixed(ctl->partials, ctl->nparts));
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
    // rounding floor: the update contracted neither by the factor `stall` nor
    // to within twice the quadratic bound ||R_{k+1}|| <= ||R_k||^2.  For
    // r >= 1/2 the bound is no contraction at all, so the loop then goes on
    // while the norm falls, however slowly.
    if (rn > fmax(stall * r, 2.0 * r * r) || it >= max_iters || rn == 0.0) ctl->run_ns = 0;
}

__global__ void refine_finish_kernel(RefineCtl *ctls, int count, double accept, int det_wanted) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= count) return;
    RefineCtl *ctl = ctls + m;
    ctl->run_ns = 0;
    if (!ctl->run_fallback) {
        if (!(ctl->r <= accept)) ctl->run_fallback = 1;
    }
    ctl->copy_back = (!ctl->run_fallback && ctl->final_buf == 1) ? 1 : 0;
    ctl->run_det = (!ctl->run_fallback && det_wanted) ? 1 : 0;
}

__device__ inline const RefMember &pick(const RefMember *mem, const RefMember &single) {
    return mem ? mem[blockIdx.x] : single;
}

__global__ void __launch_bounds__(256)
copy_back_kernel(const RefMember *mem, RefMember single, const RefineCtl *ctls) {
    const RefMember &m = pick(mem, single);
    if (!ctls[blockIdx.x].copy_back) return;
    for (int i = blockIdx.y; i < m.n; i += gridDim.y)
        for (int j = threadIdx.x; j < m.n; j += 256)
            m.X[(int64_t)i * m.ldx + j] = m.Xw[(int64_t)i * m.n + j];
}

// After the fallback run: mark its outcome.
__global__ void refine_fallback_mark_kernel(RefineCtl *ctls, int count) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= count) return;
    const RefineCtl *ctl = ctls + m;
    if (!ctl->run_fallback) return;
    if (ctl->res->code == GJ_RES_OK) ctl->res->code = GJ_RES_REFINE_FALLBACK;
    ctl->res->refine_iters = ctl->updates;
}

// Row / column order of the FP32 run as permutations: the pivoted matrix is
// B(a, b) = A(rows[a], cols[b]).  The swaps are replayed in step order (only
// where the streaming run's maps are not available).
__global__ void perms_from_pivots_kernel(const RefMember *mem, RefMember single,
                                         const RefineCtl *ctls) {
    const RefMember &m = pick(mem, single);
    if (!ctls[blockIdx.x].run_det || !m.rows_buf || threadIdx.x != 0) return;
    int32_t *rows = m.rows_buf, *cols = m.cols_buf;
    for (int i = 0; i < m.n; ++i) { rows[i] = i; cols[i] = i; }
    for (int k = 0; k < m.n; ++k) {
        const int r = m.ipiv[k], c = m.jpiv[k];
        int t = rows[k]; rows[k] = rows[r]; rows[r] = t;
        t = cols[k]; cols[k] = cols[c]; cols[c] = t;
    }
}

__global__ void __launch_bounds__(256)
gather_perm_kernel(const RefMember *mem, RefMember single, const RefineCtl *ctls) {
    const RefMember &m = pick(mem, single);
    if (!ctls[blockIdx.x].run_det) return;
    for (int a = blockIdx.y; a < m.n; a += gridDim.y) {
        const double *Ar = m.A + (int64_t)m.rows[a] * m.lda;
        for (int b = threadIdx.x; b < m.n; b += 256) m.B[(int64_t)a * m.n + b] = Ar[m.cols[b]];
    }
}

// det A = sign(P) sign(Q) prod det(S11) over the diagonal blocks.  One
// workgroup per member: its threads count the swaps of the FP32 pivot
// sequence (a serial loop over n pivots took 0.8 ms at n = 4096), then one
// thread multiplies the blocks' determinants in block order.
__global__ void __launch_bounds__(256)
det_combine_kernel(const RefMember *mem, RefMember single, RefineCtl *ctls, int count) {
    __shared__ int s_flips[256 / kWave];
    const int idx = blockIdx.x, t = threadIdx.x;
    if (idx >= count) return;
    const RefMember &m = mem ? mem[idx] : single;
    RefineCtl *ctl = ctls + idx;
    if (!ctl->run_det) return;   // the same in the whole workgroup
    int flips = 0;
    for (int k = t; k < m.n; k += 256) flips += (m.ipiv[k] != k) + (m.jpiv[k] != k);
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) flips += __shfl_xor(flips, off, kWave);
    if ((t & (kWave - 1)) == 0) s_flips[t / kWave] = flips;
    __syncthreads();
    if (t != 0) return;
    int total = 0;
    for (int w = 0; w < 256 / kWave; ++w) total += s_flips[w];
    gj_result *res = ctl->res;
    int sign = (total & 1) ? -1 : 1;
    DetAcc<double> d;
    d.init();
    bool bad = false;
    for (int b = 0; b < m.nblocks; ++b) {
        const gj_result br = m.blockres[b];
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

__global__ void refine_iters_kernel(RefineCtl *ctls, int count) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= count) return;
    if (!ctls[m].run_fallback) ctls[m].res->refine_iters = ctls[m].updates;
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
size_t refine_member_bytes() { return sizeof(RefMember); }
const int32_t *ctl_run_ns(const void *c) { return &((const RefineCtl *)c)->run_ns; }
const int32_t *ctl_run_fallback(const void *c) { return &((const RefineCtl *)c)->run_fallback; }
const int32_t *ctl_run_det(const void *c) { return &((const RefineCtl *)c)->run_det; }
const int32_t *ctl_copy_back(const void *c) { return &((const RefineCtl *)c)->copy_back; }
const int32_t *ctl_always(const void *c) { return &((const RefineCtl *)c)->always; }
void *ctl_at(void *c, int m) { return (RefineCtl *)c + m; }

#define GJ_CHECK_LAUNCH() do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)
static inline int g256(int count) { return (count + 255) / 256; }

hipError_t launch_refine_bind(void *ctl, gj_result *res, double *partials, int nparts, hipStream_t s) {
    hipLaunchKernelGGL(refine_bind_kernel, dim3(1), dim3(64), 0, s, (RefineCtl *)ctl, res, partials, nparts);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_refine_start(void *ctls, int count, hipStream_t s) {
    hipLaunchKernelGGL(refine_start_kernel, dim3(g256(count)), dim3(256), 0, s, (RefineCtl *)ctls, count);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_refine_resid0(void *ctls, int count, hipStream_t s) {
    hipLaunchKernelGGL(refine_resid0_kernel, dim3(count), dim3(256), 0, s, (RefineCtl *)ctls);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_refine_after_update(void *ctls, int count, int it, int max_iters, double stall,
                                      hipStream_t s) {
    hipLaunchKernelGGL(refine_after_update_kernel, dim3(count), dim3(256), 0, s, (RefineCtl *)ctls,
                       it, max_iters, stall);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_refine_finish(void *ctls, int count, double accept, int det_wanted, hipStream_t s) {
    hipLaunchKernelGGL(refine_finish_kernel, dim3(g256(count)), dim3(256), 0, s, (RefineCtl *)ctls,
                       count, accept, det_wanted);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_copy_back(const RefMember *mem, const RefMember &single, void *ctls, int count,
                            int row_blocks, hipStream_t s) {
    hipLaunchKernelGGL(copy_back_kernel, dim3(count, row_blocks), dim3(256), 0, s, mem, single,
                       (const RefineCtl *)ctls);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_fallback_mark(void *ctls, int count, hipStream_t s) {
    hipLaunchKernelGGL(refine_fallback_mark_kernel, dim3(g256(count)), dim3(256), 0, s,
                       (RefineCtl *)ctls, count);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_perms_from_pivots(const RefMember *mem, const RefMember &single, void *ctls,
                                    int count, hipStream_t s) {
    hipLaunchKernelGGL(perms_from_pivots_kernel, dim3(count), dim3(64), 0, s, mem, single,
                       (const RefineCtl *)ctls);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_gather_perm(const RefMember *mem, const RefMember &single, void *ctls, int count,
                              int row_blocks, hipStream_t s) {
    hipLaunchKernelGGL(gather_perm_kernel, dim3(count, row_blocks), dim3(256), 0, s, mem, single,
                       (const RefineCtl *)ctls);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_det_combine(const RefMember *mem, const RefMember &single, void *ctls, int count,
                              hipStream_t s) {
    hipLaunchKernelGGL(det_combine_kernel, dim3(count), dim3(256), 0, s, mem, single,
                       (RefineCtl *)ctls, count);
    GJ_CHECK_LAUNCH();
    return hipSuccess;
}
hipError_t launch_refine_iters(void *ctls, int count, hipStream_t s) {
    hipLaunchKernelGGL(refine_iters_kernel, dim3(g256(count)), dim3(256), 0, s, (RefineCtl *)ctls, count);
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
