// big.hip -- full-pivot Gauss-Jordan for matrices that do not fit on chip.
//
// One launch per elimination step k.  The working array W (the in-place
// [A|D] of eqs. 3-10) lives in the workspace; every step streams it once from
// HBM and back, so the sweep is HBM-bound (16 n^2 bytes per FP64 step).
//
// Layout and ownership
//   * Each workgroup owns R whole rows of W.  It reads only its own rows, the
//     pivot row and O(n) bookkeeping, and writes only its own rows.
//   * Row and column swaps (Obs. 2-3) are virtual: rows and columns stay where
//     they are and two index maps (physical -> logical position, double
//     buffered by step parity) record the permutation.  Ties in the pivot
//     search (largest |a|, lowest row, then lowest column) are decided on the
//     logical indices, i.e. on the positions in the swapped matrix.
//   * The pivot row is divided by the pivot (eq. 14) lazily: during step k every
//     workgroup reads the unscaled pivot row and divides it itself, and the
//     owner writes the scaled values one step later while applying step k+1.
//     No workgroup ever reads a row that another one is writing.
//   * The multiplier a_ik of eq. 15 comes from the workgroup's own row.
//   * The pivot search of step k+1 is fused into the sweep of step k: each
//     workgroup leaves one candidate (|a|, logical row, logical column,
//     physical row, physical column); every workgroup of step k+1 reduces the
//     whole candidate list itself, so no extra launch or grid barrier is
//     needed.
//   * The final depivoting (Obs. 3) is a gather:
//       X(i, j) = W(rowphys[collog[i]], colphys[rowlog[j]]).
#include "gj_device.h"

namespace gj {

template <typename T> struct VecOf;
template <> struct VecOf<double> { static constexpr int V = 2; using type = double2; using itype = int2; };
template <> struct VecOf<float> { static constexpr int V = 4; using type = float4; using itype = int4; };

template <typename VT, typename T>
__device__ inline T vget(const VT &x, int e) { return reinterpret_cast<const T *>(&x)[e]; }
template <typename VT, typename T>
__device__ inline void vset(VT &x, int e, T v) { reinterpret_cast<T *>(&x)[e] = v; }

constexpr int kNch = 8;  // column chunks per thread: n <= kNch * V * threads-per-row

// Workgroup-wide argmax of BigPart-like candidates, keyed on the logical
// position.  Result broadcast to every thread.
template <int NT>
__device__ inline void block_argmax(double &a, double &v, uint32_t &key, int &ip, int &jp,
                                    double *s_a, double *s_v, uint32_t *s_k, int *s_i, int *s_j) {
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) {
        double oa = __shfl_xor(a, off, kWave);
        double ov = __shfl_xor(v, off, kWave);
        uint32_t ok = (uint32_t)__shfl_xor((int)key, off, kWave);
        int oi = __shfl_xor(ip, off, kWave);
        int oj = __shfl_xor(jp, off, kWave);
        if (better(oa, ok, a, key)) { a = oa; v = ov; key = ok; ip = oi; jp = oj; }
    }
    constexpr int NW = NT / kWave;
    if constexpr (NW > 1) {
        if (lane == 0) { s_a[w] = a; s_v[w] = v; s_k[w] = key; s_i[w] = ip; s_j[w] = jp; }
        __syncthreads();
        a = s_a[0]; v = s_v[0]; key = s_k[0]; ip = s_i[0]; jp = s_j[0];
#pragma unroll
        for (int x = 1; x < NW; ++x) {
            if (better(s_a[x], s_k[x], a, key)) {
                a = s_a[x]; v = s_v[x]; key = s_k[x]; ip = s_i[x]; jp = s_j[x];
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ init
// W <- A (converted to T), identity maps, pivot candidates of step 0.
template <typename T, int NT>
__global__ void __launch_bounds__(NT)
gj_big_init(const BigDesc *__restrict__ descs, const int2 *__restrict__ bmap, const BigDesc single,
              const int32_t *__restrict__ run_flag) {
    if (run_flag && *run_flag == 0) return;
    __shared__ double s_a[NT / kWave], s_v[NT / kWave];
    __shared__ uint32_t s_k[NT / kWave];
    __shared__ int s_i[NT / kWave], s_j[NT / kWave];
    using V = VecOf<T>;
    const int2 bm = descs ? bmap[blockIdx.x] : make_int2(0, (int)blockIdx.x);
    const BigDesc d = descs ? descs[bm.x] : single;
    if (d.run && *d.run == 0) return;
    const int rb = bm.y, t = threadIdx.x, n = d.n;
    const int tpr = d.tpr, rsub = t / tpr, tc = t % tpr, rg = NT / tpr;
    T *W = reinterpret_cast<T *>(d.W);
    const int r0 = rb * d.R, r1 = min(n, r0 + d.R);
    if (rb == 0 && t == 0) { d.hdr->status = 0; d.hdr->rank = n; d.hdr->tau = 0.0; }
    if (rb == 0)
        for (int j = t; j < n; j += NT) d.collog[j] = j;
    double ba = 0.0, bv = 0.0;   // "no candidate": (0, key 0xFFFFFFFF)
    uint32_t bk = 0xFFFFFFFFu;
    int bi = -1, bj = -1;
    bool nf = false;
    for (int i = r0 + rsub; i < r1; i += rg) {
        if (tc == 0) d.rowlog[i] = i;
        for (int j = tc; j < d.ldw; j += tpr) {
            T x = (T)0;
            if (j < n) {
                x = (T)d.A[(int64_t)i * d.lda + j];
                const double ax = fabs((double)x);
                nf |= !(ax <= 1.7976931348623157e308);
                const uint32_t key = ((uint32_t)i << 16) | (uint32_t)j;
                if (better(ax, key, ba, bk)) { ba = ax; bv = (double)x; bk = key; bi = i; bj = j; }
            }
            W[(int64_t)i * d.ldw + j] = x;
        }
    }
    const int any_nf = __syncthreads_or(nf ? 1 : 0);
    block_argmax<NT>(ba, bv, bk, bi, bj, s_a, s_v, s_k, s_i, s_j);
    if (t == 0) {
        BigPart p;
        p.a = any_nf ? __builtin_inf() : ba;
        p.v = bv;
        p.rlog = (int32_t)(bk >> 16);
        p.clog = (int32_t)(bk & 0xFFFFu);
        p.iphys = bi;
        p.jphys = bj;
        d.part[rb] = p;
    }
}

// ------------------------------------------------------------------ step
template <typename T, int NT>
__global__ void __launch_bounds__(NT)
gj_big_step(const BigDesc *__restrict__ descs, const int2 *__restrict__ bmap, const BigDesc single,
            int k, double zero_tol, double eps_default, int det_only,
            const int32_t *__restrict__ run_flag) {
    if (run_flag && *run_flag == 0) return;
    using V = VecOf<T>;
    using VT = typename V::type;
    using VI = typename V::itype;
    constexpr int VE = V::V;
    __shared__ double s_a[NT / kWave], s_v[NT / kWave];
    __shared__ uint32_t s_k[NT / kWave];
    __shared__ int s_i[NT / kWave], s_j[NT / kWave];
    __shared__ T s_q[64];
    __shared__ int s_rl[64];

    const int2 bm = descs ? bmap[blockIdx.x] : make_int2(0, (int)blockIdx.x);
    const BigDesc d = descs ? descs[bm.x] : single;
    if (d.run && *d.run == 0) return;
    const int n = d.n;
    if (k >= n) return;
    if (d.hdr->status != 0) return;
    const int rb = bm.y, t = threadIdx.x;
    const int tpr = d.tpr, rsub = t / tpr, tc = t % tpr, rg = NT / tpr;
    T *W = reinterpret_cast<T *>(d.W);
    const int64_t ldw = d.ldw;
    const int r0 = rb * d.R, r1 = min(n, r0 + d.R);

    // ---- 1. reduce the candidates left by step k-1 (or the init kernel)
    double pa = 0.0, pv = 0.0;
    uint32_t pk = 0xFFFFFFFFu;
    int pi = -1, pj = -1;
    {
        const BigPart *P = d.part + (size_t)(k & 1) * d.nblk;
        for (int x = t; x < d.nblk; x += NT) {
            const BigPart c = P[x];
            const uint32_t key = ((uint32_t)c.rlog << 16) | (uint32_t)c.clog;
            if (better(c.a, key, pa, pk)) { pa = c.a; pv = c.v; pk = key; pi = c.iphys; pj = c.jphys; }
        }
        block_argmax<NT>(pa, pv, pk, pi, pj, s_a, s_v, s_k, s_i, s_j);
    }
    double tau;
    if (k == 0) {
        tau = (zero_tol >= 0.0) ? (double)(T)zero_tol : (double)((T)n * (T)eps_default * (T)pa);
        if (rb == 0 && t == 0) d.hdr->tau = tau;
    } else {
        tau = d.hdr->tau;
    }
    const bool stop_nf = !(pa <= 1.7976931348623157e308);
    // (a winner without a position cannot occur for k < n; refusing it keeps
    // every later index in bounds)
    const bool stop_sing = (pa == 0.0) || ((T)pa < (T)tau) || pi < 0 || pj < 0;
    if (stop_nf || stop_sing) {
        if (rb == 0 && t == 0) {
            d.hdr->status = stop_nf ? GJ_RES_NONFINITE : GJ_RES_SINGULAR;
            d.hdr->rank = k;
        }
        return;
    }
    const int rlog = (int)(pk >> 16), clog = (int)(pk & 0xFFFFu);
    const int rp = pi, cp = pj;
    const T p = (T)pv;
    if (rb == 0 && t == 0) {
        StepRec s;
        s.p = pv; s.rphys = rp; s.cphys = cp; s.rlog = rlog; s.clog = clog;
        d.steps[k] = s;
    }
    int rpp = -1, cpp = -1;
    T pp = (T)1;
    if (k > 0) {
        const StepRec s = d.steps[k - 1];
        rpp = s.rphys; cpp = s.cphys; pp = (T)s.p;
    }
    const T y = Num<T>::one() / p, yp = Num<T>::one() / pp;   // RN(1/p): div_pivot seeds
    const bool p_ok = div_pivot_ok(p), pp_ok = div_pivot_ok(pp);

    // ---- 2. multipliers of the owned rows (the pivot column, eq. 15) and
    //         their new logical row indices
    const int32_t *rl_old = d.rowlog + (size_t)(k & 1) * d.mstride;
    int32_t *rl_new = d.rowlog + (size_t)((k + 1) & 1) * d.mstride;
    for (int x = t; x < r1 - r0; x += NT) {
        const int i = r0 + x;
        T q = W[(int64_t)i * ldw + cp];
        if (i == rpp) q = div_pivot(q, pp, yp, pp_ok);   // deferred eq. 14 of the previous step
        s_q[x] = q;
        const int ro = rl_old[i];
        const int rn = (i == rp) ? k : ((ro == k) ? rlog : ro);
        s_rl[x] = (det_only && ro < k) ? -1 : rn;   // -1: row not needed
        rl_new[i] = rn;
    }

    // ---- 3. the pivot row divided by the pivot (eq. 14) and the new logical
    //         column indices, for this thread's columns
    const int32_t *cl_old = d.collog + (size_t)(k & 1) * d.mstride;
    int32_t *cl_new = d.collog + (size_t)((k + 1) & 1) * d.mstride;
    const int nch = (n + tpr * VE - 1) / (tpr * VE);
    const T *Wp = W + (int64_t)rp * ldw;
    T prow[kNch][VE];
    int ckey[kNch][VE];
    const T one = Num<T>::one();
#pragma unroll
    for (int c = 0; c < kNch; ++c) {
        if (c < nch) {
            const int j0 = c * tpr * VE + tc * VE;
            const VT pw = *reinterpret_cast<const VT *>(Wp + j0);
            VI co;
            if (j0 + VE <= n) {
                co = *reinterpret_cast<const VI *>(cl_old + j0);
            } else {
#pragma unroll
                for (int e = 0; e < VE; ++e) vset<VI, int>(co, e, (j0 + e < n) ? cl_old[j0 + e] : -1);
            }
#pragma unroll
            for (int e = 0; e < VE; ++e) {
                const int j = j0 + e;
                const int o = vget<VI, int>(co, e);
                const int cn = (j == cp) ? k : ((o == k) ? clog : o);
                ckey[c][e] = (j < n) ? cn : -1;
                prow[c][e] = (j == cp) ? y : div_pivot(vget<VT, T>(pw, e), p, y, p_ok);
                if (rb == 0 && rsub == 0 && j < n) cl_new[j] = cn;
            }
        } else {
#pragma unroll
            for (int e = 0; e < VE; ++e) { ckey[c][e] = -1; prow[c][e] = (T)0; }
        }
    }
    __syncthreads();

    // ---- 4. eq. 15 on the owned rows + fused pivot search for step k+1
    double ba = 0.0, bv = 0.0;   // "no candidate": (0, key 0xFFFFFFFF)
    uint32_t bk = 0xFFFFFFFFu;
    int bi = -1, bj = -1;
    bool nf = false;
    for (int x = rsub; x < r1 - r0; x += rg) {
        const int i = r0 + x;
        const int rn = s_rl[x];
        if (i == rp || rn < 0) continue;   // pivot row: written at step k+1
        const T q = s_q[x];
        const bool fix = (i == rpp);
        const bool rcand = rn > k;
        T *Wi = W + (int64_t)i * ldw;
#pragma unroll
        for (int c = 0; c < kNch; ++c) {
            if (c < nch) {
                const int j0 = c * tpr * VE + tc * VE;
                VT w = *reinterpret_cast<const VT *>(Wi + j0);
#pragma unroll
                for (int e = 0; e < VE; ++e) {
                    const int j = j0 + e;
                    T cur = vget<VT, T>(w, e);
                    if (fix) cur = (j == cpp) ? yp : div_pivot(cur, pp, yp, pp_ok);
                    if (j == cp) cur = (T)0;
                    const T nv = Num<T>::fma_(-q, prow[c][e], cur);
                    vset<VT, T>(w, e, nv);
                    const int cl = ckey[c][e];
                    if (rcand && cl > k) {
                        const double an = fabs((double)nv);
                        nf |= !(an <= 1.7976931348623157e308);
                        const uint32_t key = ((uint32_t)rn << 16) | (uint32_t)cl;
                        if (better(an, key, ba, bk)) { ba = an; bv = (double)nv; bk = key; bi = i; bj = j; }
                    }
                }
                *reinterpret_cast<VT *>(Wi + j0) = w;
            }
        }
    }
    if (k + 1 < n) {
        const int any_nf = __syncthreads_or(nf ? 1 : 0);
        block_argmax<NT>(ba, bv, bk, bi, bj, s_a, s_v, s_k, s_i, s_j);
        if (t == 0) {
            BigPart o;
            o.a = any_nf ? __builtin_inf() : ba;
            o.v = bv;
            o.rlog = (int32_t)(bk >> 16);
            o.clog = (int32_t)(bk & 0xFFFFu);
            o.iphys = bi;
            o.jphys = bj;
            d.part[(size_t)((k + 1) & 1) * d.nblk + rb] = o;
        }
    }
}

// ------------------------------------------------------------------ finish
// Inverse maps, pivot sequence, determinant and result record.
template <typename T>
__global__ void __launch_bounds__(256)
gj_big_finish(const BigDesc *__restrict__ descs, const int2 *__restrict__ bmap, const BigDesc single,
              const int32_t *__restrict__ run_flag) {
    if (run_flag && *run_flag == 0) return;
    const int2 bm = descs ? bmap[blockIdx.x] : make_int2(0, (int)blockIdx.x);
    const BigDesc d = descs ? descs[bm.x] : single;
    if (d.run && *d.run == 0) return;
    const int n = d.n, t = threadIdx.x;
    const int status = d.hdr->status;
    const int rank = (status == 0) ? n : d.hdr->rank;
    // the maps after step n-1 sit at parity n & 1
    const int32_t *rl = d.rowlog + (size_t)(n & 1) * d.mstride;
    const int32_t *cl = d.collog + (size_t)(n & 1) * d.mstride;
    const int stride = d.nblk * 256;
    for (int x = bm.y * 256 + t; x < n; x += stride) {
        if (status == 0) {
            d.rowphys[rl[x]] = x;
            d.colphys[cl[x]] = x;
        }
        if (x < rank) {
            const StepRec s = d.steps[x];
            d.ipiv[x] = s.rlog;
            d.jpiv[x] = s.clog;
        } else {
            d.ipiv[x] = -1;
            d.jpiv[x] = -1;
        }
    }
    if (bm.y == 0 && t == 0) {
        if (status == 0) {
            DetAcc<T> det;
            det.init();
            for (int k = 0; k < n; ++k) {
                const StepRec s = d.steps[k];
                det.mul((T)s.p);
                if (s.rlog != k) det.sign = -det.sign;
                if (s.clog != k) det.sign = -det.sign;
            }
            write_result_ok(d.res, n, det);
        } else {
            write_result_fail(d.res, status, rank);
        }
    }
}

// X(i, j) = W(rowphys[collog[i]], colphys[rowlog[j]]); the last pivot row
// still needs its eq. 14 division.  One workgroup per output row.
template <typename T>
__global__ void __launch_bounds__(256)
gj_big_gather(const BigDesc *__restrict__ descs, const int2 *__restrict__ bmap, const BigDesc single,
              const int32_t *__restrict__ run_flag) {
    if (run_flag && *run_flag == 0) return;
    const int2 bm = descs ? bmap[blockIdx.x] : make_int2(0, (int)blockIdx.x);
    const BigDesc d = descs ? descs[bm.x] : single;
    if (d.run && *d.run == 0) return;
    const int n = d.n, t = threadIdx.x;
    const int status = d.hdr->status;
    const T *W = reinterpret_cast<const T *>(d.W);
    const int32_t *rl = d.rowlog + (size_t)(n & 1) * d.mstride;
    const int32_t *cl = d.collog + (size_t)(n & 1) * d.mstride;
    const StepRec last = d.steps[n - 1];
    const T one = Num<T>::one();
    for (int i = bm.y; i < n; i += d.nblk) {
        double *Xi = d.X + (int64_t)i * d.ldx;
        if (status != 0) {
            for (int j = t; j < n; j += 256) Xi[j] = __builtin_nan("");
            continue;
        }
        const int src = d.rowphys[cl[i]];
        const T *Ws = W + (int64_t)src * d.ldw;
        const bool fix = (src == last.rphys);
        const T pl = (T)last.p;
        for (int j = t; j < n; j += 256) {
            const int sc = d.colphys[rl[j]];
            T x = Ws[sc];
            if (fix) x = ((sc == last.cphys) ? one : x) / pl;
            Xi[j] = (double)x;
        }
    }
}

// ---------------------------------------------------------------- launchers

template <typename T, int NT>
static hipError_t run_big_t(const BigDesc *descs, const int2 *bmap, const BigDesc &single,
                            const int *grid_per_step,
                            int grid_init, int grid_finish, int max_n, int gather_grid,
                            double zero_tol, double eps_default, int det_only, void *const *events,
                            const int32_t *run_flag, hipStream_t s) {
    hipLaunchKernelGGL((gj_big_init<T, NT>), dim3(grid_init), dim3(NT), 0, s, descs, bmap, single, run_flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (events && events[0]) {
        e = hipEventRecord((hipEvent_t)events[0], s);
        if (e != hipSuccess) return e;
    }
    for (int k = 0; k < max_n; ++k) {
        hipLaunchKernelGGL((gj_big_step<T, NT>), dim3(grid_per_step ? grid_per_step[k] : grid_init),
                           dim3(NT), 0, s, descs, bmap, single, k, zero_tol, eps_default, det_only,
                           run_flag);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (events && events[1]) {
        e = hipEventRecord((hipEvent_t)events[1], s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((gj_big_finish<T>), dim3(grid_finish), dim3(256), 0, s, descs, bmap, single, run_flag);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!det_only && gather_grid > 0) {
        hipLaunchKernelGGL((gj_big_gather<T>), dim3(gather_grid), dim3(256), 0, s, descs, bmap, single, run_flag);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_big(bool fp32, int nt, const BigDesc *descs, const int2 *bmap,
                      const BigDesc &single, const int *grid_per_step, int grid_init, int grid_finish, int max_n,
                      int gather_grid, double zero_tol, double eps_default, int det_only,
                      void *const *events, const int32_t *run_flag, hipStream_t s) {
#define GJ_BIG_CASE(TT, NTV)                                                                \
    return run_big_t<TT, NTV>(descs, bmap, single, grid_per_step, grid_init, grid_finish, max_n,   \
                              gather_grid, zero_tol, eps_default, det_only, events, run_flag, s)
    if (fp32) {
        switch (nt) {
            case 256: GJ_BIG_CASE(float, 256);
            case 512: GJ_BIG_CASE(float, 512);
            case 1024: GJ_BIG_CASE(float, 1024);
        }
    } else {
        switch (nt) {
            case 256: GJ_BIG_CASE(double, 256);
            case 512: GJ_BIG_CASE(double, 512);
            case 1024: GJ_BIG_CASE(double, 1024);
        }
    }
#undef GJ_BIG_CASE
    return hipErrorInvalidValue;
}

size_t big_part_bytes() { return sizeof(BigPart); }
size_t big_step_bytes() { return sizeof(StepRec); }
size_t big_hdr_bytes() { return sizeof(BigHdr); }
size_t big_desc_bytes() { return sizeof(BigDesc); }

}  // namespace gj
