// blocked.hip -- full-pivot Gauss-Jordan with delayed updates (FP64, and
// FP32 for the first stage of the refined path).
//
// Full pivoting only needs the trailing block S of the array: the rows and
// columns not yet eliminated (after k steps of eqs. 14-15, S is the Schur
// complement of the eliminated part, updated exactly as the unblocked
// elimination updates those positions, so the pivot sequence and the
// determinant come out bit for bit the same).  The array is kept in pivot
// order, eliminated rows and columns first, and processed in panels of nb
// steps:
//
//   1. the streaming kernels of big.hip run nb steps of the elimination on
//      S alone, in place, with their virtual row and column swaps: afterwards
//      S holds [[T, T Wb3], [-W3b T, W33 - W3b T Wb3]], T = Wbb^-1, where b
//      are the panel's pivots and 3 the rest of S;
//   2. blk_permute copies the array into the second buffer with S's rows and
//      columns in pivot order (so b follows the k0 earlier pivots), applies
//      the last pivot row's deferred eq. 14 on S's columns, and keeps copies
//      of the blocks W_b1 (rows b, earlier columns) and W_1b (earlier rows,
//      columns b), the latter zeroed in the array;
//   3. the rest of the panel's elimination is three matrix-core products
//      (the nb steps' left factors multiplied into one: by the theorem of
//      section 1 the inverse is the product of those factors, and a product
//      may be grouped):
//        W_b1 = T W_b1,  W_31 += W_3b W_b1(old),  W_1* -= W_1b(old) W_b*.
//
// Each step then streams (n - k0)^2 elements instead of n^2, about a third of
// the bytes over a whole inversion; the products touch the remaining
// columns once per panel.  The inverse differs from the unblocked one by
// rounding only (the products sum in another order).  At the end
//   X(i, j) = W(colinv[i], rowinv[j]),
// with rowinv and colinv the positions of the original rows and columns.
#include "gj_launch.h"

namespace gj {

namespace {

__global__ void __launch_bounds__(256)
blk_init_perm(int32_t *prow, int32_t *pcol, int n) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x < n) { prow[x] = x; pcol[x] = x; }
}

// After a panel of nbp steps on the trailing block of order m (steps k0 ..
// k0 + nbp - 1): logical -> physical maps of the block, and the panel's step
// records with global logical positions (only the steps that ran when the
// elimination stopped inside the panel).
__global__ void __launch_bounds__(256)
blk_panel_maps(const BigHdr *__restrict__ hdr, const int32_t *__restrict__ rl,
               const int32_t *__restrict__ cl, int m, int32_t *__restrict__ rphys,
               int32_t *__restrict__ cphys, StepRec *__restrict__ steps, int nbp, int k0) {
    const int status = hdr->status;
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int done = status == 0 ? nbp : max(0, min(nbp, hdr->rank - k0));
    if (x < done) {
        steps[x].rlog += k0;
        steps[x].clog += k0;
    }
    if (status != 0 || x >= m) return;
    rphys[rl[x]] = x;
    cphys[cl[x]] = x;
}

// One workgroup per destination row r: W2(r, c) = W(src(r), src(c)), where
// rows and columns before k0 stay and the block's follow rphys / cphys.
// Columns from n to ldw are zeroed (the block's row shape may reach them).
template <typename T>
__global__ void __launch_bounds__(256)
blk_permute(const BigHdr *__restrict__ hdr, const T *__restrict__ W, T *__restrict__ W2,
            int64_t ldw, int n, int k0, int nbp, const int32_t *__restrict__ rphys,
            const int32_t *__restrict__ cphys, const StepRec *__restrict__ last,
            T *__restrict__ tA, int ldta, T *__restrict__ tB, int64_t ldtb,
            const int32_t *__restrict__ prow_old, const int32_t *__restrict__ pcol_old,
            int32_t *__restrict__ prow_new, int32_t *__restrict__ pcol_new) {
    if (hdr->status != 0) return;
    const int r = blockIdx.x, t = threadIdx.x;
    const int sr = r < k0 ? r : k0 + rphys[r - k0];
    const StepRec ls = *last;
    const int lc = k0 + ls.cphys;
    const bool fix = sr == k0 + ls.rphys;   // the last pivot row: its eq. 14 on the block's columns
    const T lp = (T)ls.p;   // the pivot, exact in T (the elimination's own value)
    const T *Ws = W + (int64_t)sr * ldw;
    T *Wd = W2 + (int64_t)r * ldw;
    const bool in_b = r >= k0 && r < k0 + nbp;
    for (int c = t; c < ldw; c += 256) {
        T x = (T)0;
        if (c < n) {
            const int sc = c < k0 ? c : k0 + cphys[c - k0];
            x = Ws[sc];
            if (fix && sc >= k0) x = ((sc == lc) ? (T)1 : x) / lp;
            if (in_b && c < k0) tB[(int64_t)(r - k0) * ldtb + c] = x;
            if (r < k0 && c >= k0 && c < k0 + nbp) {
                tA[(int64_t)r * ldta + (c - k0)] = x;
                x = (T)0;
            }
        }
        Wd[c] = x;
    }
    if (t == 0) prow_new[r] = prow_old[sr];
    if (r == 0)
        for (int c = t; c < n; c += 256) pcol_new[c] = pcol_old[c < k0 ? c : k0 + cphys[c - k0]];
}

// Pivot sequence, determinant (eq. 13, the product of the pivots in step
// order, as the unblocked elimination forms it) and result record; inverse
// position maps for the gather.
__global__ void __launch_bounds__(256)
blk_finish(const BigHdr *__restrict__ hdr, const StepRec *__restrict__ steps, int n,
           int32_t *__restrict__ ipiv, int32_t *__restrict__ jpiv, gj_result *__restrict__ res,
           const int32_t *__restrict__ prow, const int32_t *__restrict__ pcol,
           int32_t *__restrict__ rowinv, int32_t *__restrict__ colinv) {
    const int status = hdr->status;
    const int rank = (status == 0) ? n : hdr->rank;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x < n) {
        if (status == 0) {
            rowinv[prow[x]] = x;
            colinv[pcol[x]] = x;
        }
        if (x < rank) {
            ipiv[x] = steps[x].rlog;
            jpiv[x] = steps[x].clog;
        } else {
            ipiv[x] = -1;
            jpiv[x] = -1;
        }
    }
    if (blockIdx.x != 0) return;
    // the product runs on one thread in step order; the records pass through
    // LDS in chunks, so that it does not wait on global memory at every step
    constexpr int kChunk = 1024;
    __shared__ double s_p[kChunk];
    __shared__ int s_flip[kChunk];
    DetAcc<double> det;
    det.init();
    for (int b0 = 0; status == 0 && b0 < n; b0 += kChunk) {
        const int cnt = min(kChunk, n - b0);
        for (int y = threadIdx.x; y < cnt; y += 256) {
            const StepRec s = steps[b0 + y];
            s_p[y] = s.p;
            s_flip[y] = (s.rlog != b0 + y) ^ (s.clog != b0 + y);
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int y = 0; y < cnt; ++y) {
                det.mul(s_p[y]);
                if (s_flip[y]) det.sign = -det.sign;
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (status == 0)
            write_result_ok(res, n, det);
        else
            write_result_fail(res, status, rank);
    }
}

// X(i, j) = W(colinv[i], rowinv[j]); NaN when the elimination stopped.
template <typename T>
__global__ void __launch_bounds__(256)
blk_gather(const BigHdr *__restrict__ hdr, const T *__restrict__ W, int64_t ldw, int n,
           const int32_t *__restrict__ rowinv, const int32_t *__restrict__ colinv,
           double *__restrict__ X, int64_t ldx) {
    const int status = hdr->status;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        double *Xi = X + (int64_t)i * ldx;
        if (status != 0) {
            for (int j = threadIdx.x; j < n; j += 256) Xi[j] = __builtin_nan("");
            continue;
        }
        const T *Ws = W + (int64_t)colinv[i] * ldw;
        for (int j = threadIdx.x; j < n; j += 256) Xi[j] = (double)Ws[rowinv[j]];
    }
}

}  // namespace

hipError_t launch_blk_init_perm(int32_t *prow, int32_t *pcol, int n, hipStream_t s) {
    hipLaunchKernelGGL(blk_init_perm, dim3((n + 255) / 256), dim3(256), 0, s, prow, pcol, n);
    return hipGetLastError();
}

hipError_t launch_blk_panel_end(bool fp32, const BigHdr *hdr, const int32_t *rl, const int32_t *cl,
                                int m, int32_t *rphys, int32_t *cphys, StepRec *steps_k0, int nbp,
                                int k0, const void *W, void *W2, int64_t ldw, int n, void *tA,
                                int ldta, void *tB, int64_t ldtb, const int32_t *prow_old,
                                const int32_t *pcol_old, int32_t *prow_new, int32_t *pcol_new,
                                hipStream_t s) {
    hipLaunchKernelGGL(blk_panel_maps, dim3((m + 255) / 256), dim3(256), 0, s, hdr, rl, cl, m, rphys,
                       cphys, steps_k0, nbp, k0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (fp32)
        hipLaunchKernelGGL(blk_permute<float>, dim3(n), dim3(256), 0, s, hdr, (const float *)W,
                           (float *)W2, ldw, n, k0, nbp, rphys, cphys, steps_k0 + (nbp - 1),
                           (float *)tA, ldta, (float *)tB, ldtb, prow_old, pcol_old, prow_new,
                           pcol_new);
    else
        hipLaunchKernelGGL(blk_permute<double>, dim3(n), dim3(256), 0, s, hdr, (const double *)W,
                           (double *)W2, ldw, n, k0, nbp, rphys, cphys, steps_k0 + (nbp - 1),
                           (double *)tA, ldta, (double *)tB, ldtb, prow_old, pcol_old, prow_new,
                           pcol_new);
    return hipGetLastError();
}

hipError_t launch_blk_finish(bool fp32, const BigHdr *hdr, const StepRec *steps, int n,
                             int32_t *ipiv, int32_t *jpiv, gj_result *res, const int32_t *prow,
                             const int32_t *pcol, int32_t *rowinv, int32_t *colinv, const void *W,
                             int64_t ldw, double *X, int64_t ldx, hipStream_t s) {
    hipLaunchKernelGGL(blk_finish, dim3((n + 255) / 256), dim3(256), 0, s, hdr, steps, n, ipiv, jpiv,
                       res, prow, pcol, rowinv, colinv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !X) return e;
    if (fp32)
        hipLaunchKernelGGL(blk_gather<float>, dim3(std::min(n, 4096)), dim3(256), 0, s, hdr,
                           (const float *)W, ldw, n, rowinv, colinv, X, ldx);
    else
        hipLaunchKernelGGL(blk_gather<double>, dim3(std::min(n, 4096)), dim3(256), 0, s, hdr,
                           (const double *)W, ldw, n, rowinv, colinv, X, ldx);
    return hipGetLastError();
}

}  // namespace gj
