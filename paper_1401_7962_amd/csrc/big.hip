// big.hip -- full-pivot Gauss-Jordan for matrices that do not fit on chip.
//
// One launch per elimination step k.  The working array W (the in-place
// [A|D] of eqs. 3-10) lives in the workspace; every step streams it once from
// HBM and back, so the sweep is HBM-bound (16 n^2 bytes per FP64 step).
//
// Layout and ownership
//   * A step sweeps W in work units of whole rows (as many rows as a
//     workgroup holds in registers at once).  Each workgroup takes a few
//     units by its index, then asks a per-step counter for more until none
//     are left: on MI355X some XCDs stream measurably slower than others, and
//     a fixed split would make every step wait for the slowest.  A unit is
//     read and written only by the workgroup that took it; besides it, a
//     workgroup reads the pivot row and O(n) bookkeeping.
//   * Row and column swaps (Obs. 2-3) are virtual: rows and columns stay where
//     they are and two index maps (physical -> logical position, double
//     buffered by step parity) record the permutation.  Ties in the pivot
//     search (largest |a|, lowest row, then lowest column) are decided on the
//     logical indices, i.e. on the positions in the swapped matrix.
//   * The pivot row is divided by the pivot (eq. 14) lazily: during step k every
//     workgroup reads the unscaled pivot row and divides it itself, and the
//     workgroup that sweeps it at step k+1 writes the scaled values while
//     applying that step.  No workgroup ever reads a row that another one is
//     writing.
//   * The multiplier a_ik of eq. 15 is read from the row before the sweep of
//     its unit starts (the sweep overwrites it).
//   * The pivot search of step k+1 is fused into the sweep of step k: each
//     workgroup leaves one candidate (|a|, logical row, logical column,
//     physical row, physical column); every workgroup of step k+1 reduces the
//     whole candidate list itself, so no extra launch or grid barrier is
//     needed.
//   * The final depivoting (Obs. 3) is a gather:
//       X(i, j) = W(rowphys[collog[i]], colphys[rowlog[j]]).
//   * Other pivot rules (d.rule): 1 partial pivoting on |a| (largest |a| in
//     the next column), 2 the rule of the program in section 3 (the row with
//     the largest positive value in the next column, else the next row).
//     Both only restrict the candidates to one column; no column moves.
//   * Solving A X = B runs the same elimination on [A | B] (eq. 2 with
//     D^0 = B): the m columns of B follow A's columns in W (from column
//     rhs0: n, or the end of A's last register chunk), get the same eq. 14-15
//     updates and are never pivot candidates.  The column swaps of A come
//     back as row swaps of the result: X(i, j) = W(rowphys[collog[i]], rhs0 + j).
//   * The blocked elimination (blocked.hip) runs these kernels on the
//     trailing block of a larger array for a few steps at a time: W then
//     points into that array, d.k0 counts the steps already taken (the zero
//     threshold and the rank are global) and d.inplace makes the init kernel
//     read the block where it is and keep the header.
#include <type_traits>

#include "gj_device.h"

namespace gj {

template <typename T> struct VecOf;
template <> struct VecOf<double> { static constexpr int V = 2; using type = double2; using itype = int2; };
template <> struct VecOf<float> { static constexpr int V = 4; using type = float4; using itype = int4; };

// Row traffic of the working array (one 16-byte vector per access).  With
// NTL the loads and stores are nontemporal: once the swept array is larger
// than the Infinity Cache nothing read or written in a step is used again
// before it is evicted (with the stores too, 8192^2 FP64 steps run 9% faster;
// a cache-resident array runs 2-6% slower with them).
template <typename VT> struct NVec;
template <> struct NVec<double2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct NVec<float4> { typedef float type __attribute__((ext_vector_type(4))); };
template <bool NTL, typename VT> __device__ __forceinline__ VT row_ld(gptr<const VT> p) {
    if constexpr (NTL) {
        using NV = typename NVec<VT>::type;
        const NV nv = __builtin_nontemporal_load(reinterpret_cast<gptr<const NV>>(p));
        VT v;
        __builtin_memcpy(&v, &nv, sizeof(NV));
        return v;
    } else {
        return *p;
    }
}
template <bool NTL, typename VT> __device__ __forceinline__ void row_st(gptr<VT> p, const VT &v) {
    if constexpr (NTL) {
        using NV = typename NVec<VT>::type;
        NV nv;
        __builtin_memcpy(&nv, &v, sizeof(NV));
        __builtin_nontemporal_store(nv, reinterpret_cast<gptr<NV>>(p));
    } else {
        *p = v;
    }
}

template <typename VT, typename T>
__device__ inline T vget(const VT &x, int e) { return reinterpret_cast<const T *>(&x)[e]; }
template <typename VT, typename T>
__device__ inline void vset(VT &x, int e, T v) { reinterpret_cast<T *>(&x)[e] = v; }

// Column chunks per thread of the step kernel (its NCH): n <= NCH * V * threads-per-row.
// 8 in general; a shape whose rows fill exactly 1-7 chunks per thread gets a kernel
// of that many, whose loops and register arrays then hold no unused chunk.
constexpr int kNch = 8;
// Rows a thread holds in registers at once in the step kernel (their loads
// are in flight together; the first group is requested before the candidate
// reduction).  The 1024-thread workgroups have 128 VGPRs per lane: they load
// each chunk where it is used.
template <int NT> constexpr bool kEarlyRows = NT < 1024;
template <int NT> constexpr int kRowGroup = kEarlyRows<NT> ? 2 : 1;
// Rows per workgroup of the step kernel (its own units) are at most this many.
constexpr int kMaxUnit = 64;

// Wavefront argmax of (a, v, key, pos) candidates without LDS: DPP moves
// within rows of 16 lanes, then permlane swaps across rows (gfx950).  pos
// packs the physical position (row << 16 | column, 0xFFFF for -1).
struct BigCand {
    double a, v;
    uint32_t key, pos;
};
__device__ __forceinline__ void bigcand_take(BigCand &c, const BigCand &o) {
    if (better(o.a, o.key, c.a, c.key)) c = o;
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const uint32_t lo = dpp_u32<CTRL>((uint32_t)__double2loint(x));
    const uint32_t hi = dpp_u32<CTRL>((uint32_t)__double2hiint(x));
    return __hiloint2double((int)hi, (int)lo);
}
template <int CTRL>
__device__ __forceinline__ void bigcand_dpp(BigCand &c) {
    BigCand o;
    o.a = dpp_f64<CTRL>(c.a);
    o.v = dpp_f64<CTRL>(c.v);
    o.key = dpp_u32<CTRL>(c.key);
    o.pos = dpp_u32<CTRL>(c.pos);
    bigcand_take(c, o);
}
// permlane{16,32}_swap leave the pair in the same order in both lanes, so
// combining the two halves gives both lanes the same winner
template <bool P32>
__device__ __forceinline__ void bigcand_perm(BigCand &c) {
    uint32_t w[6] = {(uint32_t)__double2loint(c.a), (uint32_t)__double2hiint(c.a),
                     (uint32_t)__double2loint(c.v), (uint32_t)__double2hiint(c.v), c.key, c.pos};
    uint32_t x[6], y[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        auto pr = P32 ? __builtin_amdgcn_permlane32_swap(w[e], w[e], false, false)
                      : __builtin_amdgcn_permlane16_swap(w[e], w[e], false, false);
        x[e] = pr[0];
        y[e] = pr[1];
    }
    BigCand cx, cy;
    cx.a = __hiloint2double((int)x[1], (int)x[0]); cx.v = __hiloint2double((int)x[3], (int)x[2]);
    cx.key = x[4]; cx.pos = x[5];
    cy.a = __hiloint2double((int)y[1], (int)y[0]); cy.v = __hiloint2double((int)y[3], (int)y[2]);
    cy.key = y[4]; cy.pos = y[5];
    bigcand_take(cx, cy);
    c = cx;
}

// Workgroup-wide argmax of BigPart-like candidates, keyed on the logical
// position.  Result broadcast to every thread.
template <int NT>
__device__ inline void block_argmax(double &a, double &v, uint32_t &key, int &ip, int &jp,
                                    double *s_a, double *s_v, uint32_t *s_k, int *s_i, int *s_j) {
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    BigCand c;
    c.a = a; c.v = v; c.key = key;
    c.pos = ((uint32_t)(ip & 0xFFFF) << 16) | (uint32_t)(jp & 0xFFFF);
    bigcand_dpp<0xB1>(c);    // quad_perm [1,0,3,2]
    bigcand_dpp<0x4E>(c);    // quad_perm [2,3,0,1]
    bigcand_dpp<0x141>(c);   // row_half_mirror
    bigcand_dpp<0x140>(c);   // row_mirror
    bigcand_perm<false>(c);
    bigcand_perm<true>(c);
    a = c.a; v = c.v; key = c.key;
    ip = (c.pos >> 16) == 0xFFFFu ? -1 : (int)(c.pos >> 16);
    jp = (c.pos & 0xFFFFu) == 0xFFFFu ? -1 : (int)(c.pos & 0xFFFFu);
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
    if (rb == 0 && t == 0) {
        if (!d.inplace) { d.hdr->status = 0; d.hdr->rank = n; d.hdr->tau = 0.0; }
        d.hdr->ticket[0] = 0; d.hdr->ticket[1] = 0;
    }
    if (rb == 0)
        for (int j = t; j < n; j += NT) d.collog[j] = j;
    double ba = 0.0, bv = 0.0;   // "no candidate": (0, key 0xFFFFFFFF)
    uint32_t bk = 0xFFFFFFFFu;
    int bi = -1, bj = -1;
    bool nf = false;
    for (int i = r0 + rsub; i < r1; i += rg) {
        if (tc == 0) d.rowlog[i] = i;
        // in place: only the block's own columns (the row stride reaches
        // past them into the rest of the array)
        for (int j = tc; j < (d.inplace ? n : d.ldw); j += tpr) {
            T x = (T)0;
            if (j >= d.rhs0 && j < d.ncol) x = (T)d.B[(int64_t)i * d.ldb + (j - d.rhs0)];   // solve: D^0 = B
            if (j < n) {
                x = d.inplace ? W[(int64_t)i * d.ldw + j] : (T)d.A[(int64_t)i * d.lda + j];
                const double ax = fabs((double)x);
                // candidates: the whole matrix, or column 0 for the other
                // rules; the program's rule scores the value itself and takes
                // row 0 (score 0) when nothing in the column is positive
                const bool incol = d.rule == 0 || j == 0;
                nf |= incol && !(ax <= 1.7976931348623157e308);
                const double sc = d.rule == 2 ? (x > (T)0 ? (double)x : 0.0) : ax;
                const bool cand = incol && (d.rule != 2 || x > (T)0 || i == 0);
                const uint32_t key = ((uint32_t)i << 16) | (uint32_t)j;
                if (cand && better(sc, key, ba, bk)) { ba = sc; bv = (double)x; bk = key; bi = i; bj = j; }
            }
            if (!d.inplace) W[(int64_t)i * d.ldw + j] = x;
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
// FULL: every matrix of the launch uses all NCH chunks per thread (the
// chunk tests then fold away; they cost about 8% at n = 4096).
// CNT: some units may come from the per-step counter.  Without it each
// workgroup sweeps only its own rows, with no barrier in the sweep.
// RULE: the pivot rule (d.rule); 1 and 2 restrict the candidates to the
// next column, 2 scores the signed value.
// RHS: a solve whose A fills all NCH = 8 chunks; B's m columns sit after them,
// from column rhs0 = 8 * tpr * VE, as a partial extra chunk held by the
// first ceil(m / VE) threads of each row (FULL, 256/512 threads only).
template <typename T, int NT, bool NTL, bool FULL, bool CNT, bool RHS, int RULE, int NCH>
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
    __shared__ T s_qs[kMaxUnit], s_qd[2][kMaxUnit];   // multipliers: own rows, counted units
    __shared__ int s_rls[kMaxUnit], s_rld[2][kMaxUnit];  // new logical row indices (-1: skip)
    __shared__ int s_nx[2], s_first;

    const int2 bm = descs ? bmap[blockIdx.x] : make_int2(0, (int)blockIdx.x);
    const BigDesc d = descs ? descs[bm.x] : single;
    const int n = d.n;
    if (k >= n) return;
    if (d.run && *glb(d.run) == 0) return;
    const int rb = bm.y, t = threadIdx.x;
    const int tpr = d.tpr, rsub = t / tpr, tc = t % tpr, rg = NT / tpr;
    const gptr<T> W = glb(reinterpret_cast<T *>(d.W));
    const int64_t ldw = d.ldw;
    static_assert(!RHS || (FULL && kEarlyRows<NT>), "the extra chunk needs the full register layout");
    const int nch = RHS ? NCH : (d.ncol + tpr * VE - 1) / (tpr * VE);   // chunks holding A's (and B's) columns
    const int nrc = RHS ? (d.ncol - d.rhs0 + VE - 1) / VE : 1;   // threads of a row holding B
    const int bcol = d.rhs0 + min(tc, nrc - 1) * VE;            // this thread's B columns (clamped)
    const bool bown = tc < nrc;
    const gptr<BigHdr> hdr = glb(d.hdr);
    const gptr<const int32_t> rl_old = glb(static_cast<const int32_t *>(d.rowlog)) + (size_t)(k & 1) * d.mstride;
    const gptr<int32_t> rl_new = glb(d.rowlog) + (size_t)((k + 1) & 1) * d.mstride;
    const gptr<const int32_t> cl_old = glb(static_cast<const int32_t *>(d.collog)) + (size_t)(k & 1) * d.mstride;
    const gptr<int32_t> cl_new = glb(d.collog) + (size_t)((k + 1) & 1) * d.mstride;

    // The step's critical path is: candidate list -> reduction -> pivot row
    // -> scaled pivot row -> sweep.  Everything that does not depend on the
    // winner is requested up front, next to the candidates: the header, the
    // previous step's record, and the index maps of the owned rows and
    // columns.  The memory counter retires in order and the compiler can only
    // count loads that are issued on every path, so loads are unconditional
    // with clamped addresses wherever a later wait must not cover them.
    const int status = hdr->status;
    const double tau_prev = hdr->tau;
    StepRec prev;
    prev.p = 1.0; prev.rphys = -1; prev.cphys = -1;
    if (k > 0) prev = glb(d.steps)[k - 1];
    const gptr<const BigPart> P = glb(static_cast<const BigPart *>(d.part)) + (size_t)(k & 1) * d.nblk;
    const BigPart c0 = P[min(t, d.nblk - 1)];
    // Work units: one register group of rows (B * rg rows).  Units
    // [rb*S, rb*S+S) are this workgroup's; when the workgroups' units do not
    // cover the matrix, the rest are handed out by a per-step counter.
    constexpr int B = kRowGroup<NT>;
    const int U = min(B * rg, d.R);                // rows per unit; slots x >= U are unused
    const int nunits = (n + U - 1) / U;
    const int S = d.ustat;                         // S * U <= R <= kMaxUnit
    const int s0 = rb * S;
    const int nstat = max(0, min(S, nunits - s0));
    const int r0 = s0 * U;                         // the workgroup's own rows: [r0, r0 + nsr)
    const int nsr = nstat > 0 ? min(nstat * U, n - r0) : 0;
    const int dyn0 = d.nblk * S;                   // first unit of the counter
    const bool dyn = CNT && dyn0 < nunits;         // (then every workgroup has S units)
    const int ro_own = rl_old[nsr > 0 ? r0 + min(t, nsr - 1) : 0];   // old logical index of own row t
    VI co[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c)   // in bounds: the maps hold ldw >= nch * tpr * VE entries
        co[c] = *reinterpret_cast<gptr<const VI>>(cl_old + (c < nch ? c : 0) * tpr * VE + tc * VE);

    // ---- 1. reduce the candidates left by step k-1 (or the init kernel)
    double pa = 0.0, pv = 0.0;
    uint32_t pk = 0xFFFFFFFFu;
    int pi = -1, pj = -1;
    for (int x = t + NT; x < d.nblk; x += NT) {   // more workgroups than threads
        const BigPart c = P[x];
        const uint32_t key = ((uint32_t)c.rlog << 16) | (uint32_t)c.clog;
        if (better(c.a, key, pa, pk)) { pa = c.a; pv = c.v; pk = key; pi = c.iphys; pj = c.jphys; }
    }
    if (status != 0) return;
    if (t < d.nblk) {
        // the fold order does not matter: candidates of different
        // workgroups have different keys
        const uint32_t key = ((uint32_t)c0.rlog << 16) | (uint32_t)c0.clog;
        if (better(c0.a, key, pa, pk)) { pa = c0.a; pv = c0.v; pk = key; pi = c0.iphys; pj = c0.jphys; }
    }
    block_argmax<NT>(pa, pv, pk, pi, pj, s_a, s_v, s_k, s_i, s_j);
    double tau;
    if (k == 0 && d.k0 == 0) {
        // preset threshold: n eps max|a| for the text's rule, none (0) for the
        // others (the program has none)
        tau = (zero_tol >= 0.0) ? (double)(T)zero_tol
                                : (RULE == 0 ? (double)((T)n * (T)eps_default * (T)pa) : 0.0);
        if (rb == 0 && t == 0) hdr->tau = tau;
    } else {
        tau = tau_prev;
    }
    const bool stop_nf = !(pa <= 1.7976931348623157e308);
    // (a winner without a position cannot occur for k < n; refusing it keeps
    // every later index in bounds)
    const double apv = fabs(pv);   // |pivot| (the winner's score is |pv| for RULE < 2)
    const bool stop_sing = (apv == 0.0) || ((T)apv < (T)tau) || pi < 0 || pj < 0;
    if (stop_nf || stop_sing) {
        if (rb == 0 && t == 0) {
            hdr->status = stop_nf ? GJ_RES_NONFINITE : GJ_RES_SINGULAR;
            hdr->rank = d.k0 + k;
        }
        return;
    }
    const int rlog = (int)(pk >> 16), clog = (int)(pk & 0xFFFFu);
    const int rp = pi, cp = pj;
    const T p = (T)pv;

    // ---- 2. the winner's row, the own rows' multipliers (eq. 15), then the
    //         first group of own rows
    const gptr<const T> Wp = W + (int64_t)rp * ldw;
    VT pw[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c)
        pw[c] = *reinterpret_cast<gptr<const VT>>(Wp + (c < nch ? c : 0) * tpr * VE + tc * VE);
    VT pwb;
    if constexpr (RHS) pwb = *reinterpret_cast<gptr<const VT>>(Wp + bcol);
    // (slots without a row read the pivot row, which nobody writes this step)
    T q_own = W[(int64_t)(nsr > 0 ? r0 + min(t, nsr - 1) : rp) * ldw + cp];
    VT wb[B][NCH];
    VT wbb[B];   // RHS: the B chunk of each row slot
    const bool early = kEarlyRows<NT> && !det_only;
    if constexpr (kEarlyRows<NT>) {
        // rows not owned, the pivot row (written at step k+1) and every row
        // in det_only mode read the pivot row instead, and are not used
#pragma unroll
        for (int g = 0; g < B; ++g) {
            const int x = rsub + g * rg;
            const bool use = early && x < min(U, nsr) && r0 + x != rp;
            const gptr<const T> Wi = W + (int64_t)(use ? r0 + x : rp) * ldw;
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                wb[g][c] = row_ld<NTL>(reinterpret_cast<gptr<const VT>>(Wi + (c < nch ? c : 0) * tpr * VE + tc * VE));
            if constexpr (RHS) wbb[g] = row_ld<NTL>(reinterpret_cast<gptr<const VT>>(Wi + bcol));
        }
    }
    if (rb == 0 && t == 0) {
        StepRec s;
        s.p = pv; s.rphys = rp; s.cphys = cp; s.rlog = rlog; s.clog = clog;
        glb(d.steps)[k] = s;
        __hip_atomic_store(&hdr->ticket[(k + 1) & 1], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const int rpp = prev.rphys, cpp = prev.cphys;
    const T pp = (T)prev.p;
    const T y = Num<T>::one() / p, yp = Num<T>::one() / pp;   // RN(1/p): div_pivot seeds
    const bool p_ok = div_pivot_ok(p), pp_ok = div_pivot_ok(pp);

    // multiplier (with the previous pivot row's deferred eq. 14) and new
    // logical index of row i, whose old logical index is ro
    auto row_meta = [&](int i, T qraw, int ro, T *sq, int *srl, int x) {
        T q = qraw;
        if (i == rpp) q = div_pivot(q, pp, yp, pp_ok);
        const int rn = (i == rp) ? k : ((ro == k) ? rlog : ro);
        sq[x] = q;
        srl[x] = (det_only && ro < k) ? -1 : rn;   // -1: row not needed
        rl_new[i] = rn;
    };
    if (t < nsr) row_meta(r0 + t, q_own, ro_own, s_qs, s_rls, t);

    // ---- 3. the pivot row divided by the pivot (eq. 14) and the new logical
    //         column indices, for this thread's columns
    T prow[NCH][VE];
    int ckey[NCH][VE];
    bool slow = false;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int j0 = c * tpr * VE + tc * VE;
        if (FULL || c < nch) {   // the same for the whole workgroup: a scalar branch
#pragma unroll
            for (int e = 0; e < VE; ++e) {
                const int j = j0 + e;
                const int o = vget<VI, int>(co[c], e);
                const int cn = (j == cp) ? k : ((o == k) ? clog : o);
                ckey[c][e] = (j < n) ? cn : -1;
                const T qd = div_pivot_fast(vget<VT, T>(pw[c], e), p, y, p_ok, slow);
                prow[c][e] = (j == cp) ? y : qd;
            }
        } else {
#pragma unroll
            for (int e = 0; e < VE; ++e) { ckey[c][e] = -1; prow[c][e] = (T)0; }
        }
    }
    T prowb[VE];   // RHS: the pivot row's B columns divided by the pivot
    if constexpr (RHS) {
#pragma unroll
        for (int e = 0; e < VE; ++e) prowb[e] = div_pivot_fast(vget<VT, T>(pwb, e), p, y, p_ok, slow);
    }
    if (slow) {   // operands outside the corrected-quotient range: IEEE division
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int e = 0; e < VE; ++e) {
                const int j = c * tpr * VE + tc * VE + e;
                if (c < nch && j != cp) prow[c][e] = div_pivot(vget<VT, T>(pw[c], e), p, y, p_ok);
            }
        if constexpr (RHS) {
#pragma unroll
            for (int e = 0; e < VE; ++e) prowb[e] = div_pivot(vget<VT, T>(pwb, e), p, y, p_ok);
        }
    }
    if (rb == 0 && rsub == 0) {
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int e = 0; e < VE; ++e) {
                const int j = c * tpr * VE + tc * VE + e;
                if (c < nch && j < n) cl_new[j] = ckey[c][e];
            }
    }
    __syncthreads();

    // ---- 4. eq. 15 on the swept rows + fused pivot search for step k+1
    T bvT = (T)0;                 // running best (signed), "no candidate": (0, key 0xFFFFFFFF)
    T bsT = (T)-1;                // RULE 2: the best's score (-1: no candidate)
    uint32_t bk = 0xFFFFFFFFu;
    int bi = -1, bj = -1;
    bool nf = false;
    // one row already in wb[g] (or, with 1024 threads, read chunk by chunk)
    auto sweep_row = [&](int g, int i, T q, int rn) {
        const bool fix = (i == rpp);
        const bool rcand = rn > k;
        const uint32_t rkey = (uint32_t)rn << 16;
        const gptr<T> Wi = W + (int64_t)i * ldw;
        // eq. 15 for one element, then the branch-free candidate update
        // (nearly every lane takes part, so selects beat branches)
        auto update = [&](T cur, int c, int e, int j) -> T {
            cur = (j == cp) ? (T)0 : cur;
            const T nv = Num<T>::fma_(-q, prow[c][e], cur);
            const int cl = ckey[c][e];
            // '&', '|': no short-circuit branches
            const bool cand = rcand & (RULE == 0 ? (cl > k) : (cl == k + 1));
            const T an = Num<T>::abs_(nv);
            nf |= cand & !Num<T>::finite_(an);
            const uint32_t key = rkey | (uint32_t)cl;
            bool upd;
            if constexpr (RULE == 2) {   // largest positive value, else the next row (score 0)
                const T sc = (nv > (T)0) ? nv : ((rn == k + 1) ? (T)0 : (T)-1);
                upd = cand & (sc >= (T)0) & ((sc > bsT) | ((sc == bsT) & (key < bk)));
                bsT = upd ? sc : bsT;
            } else {
                const T ab = Num<T>::abs_(bvT);   // in T: exact
                upd = cand & ((an > ab) | ((an == ab) & (key < bk)));
            }
            bvT = upd ? nv : bvT;
            bk = upd ? key : bk;
            bi = upd ? i : bi;
            bj = upd ? j : bj;
            return nv;
        };
        if constexpr (kEarlyRows<NT>) {
            if (fix) {   // the previous pivot row: its deferred eq. 14 first
#pragma unroll
                for (int c = 0; c < NCH; ++c)
#pragma unroll
                    for (int e = 0; e < VE; ++e) {
                        const int j = c * tpr * VE + tc * VE + e;
                        const T cur = vget<VT, T>(wb[g][c], e);
                        vset<VT, T>(wb[g][c], e, (j == cpp) ? yp : div_pivot(cur, pp, yp, pp_ok));
                    }
            }
            // the whole row is updated in place in wb before any of it is
            // stored: a store's data registers cannot be reused until the
            // store has completed, so a register shared by all chunks would
            // serialise them
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                if (FULL || c < nch)
#pragma unroll
                    for (int e = 0; e < VE; ++e)
                        vset<VT, T>(wb[g][c], e,
                                    update(vget<VT, T>(wb[g][c], e), c, e, c * tpr * VE + tc * VE + e));
            if constexpr (RHS) {   // B's columns: eqs. 14-15 as for A's, never candidates
#pragma unroll
                for (int e = 0; e < VE; ++e) {
                    T cur = vget<VT, T>(wbb[g], e);
                    if (fix) cur = div_pivot(cur, pp, yp, pp_ok);
                    vset<VT, T>(wbb[g], e, Num<T>::fma_(-q, prowb[e], cur));
                }
            }
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                if (FULL || c < nch) row_st<NTL>(reinterpret_cast<gptr<VT>>(Wi + c * tpr * VE + tc * VE), wb[g][c]);
            if constexpr (RHS)
                if (bown) row_st<NTL>(reinterpret_cast<gptr<VT>>(Wi + bcol), wbb[g]);
        } else {
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                if (c < nch) {
                    const int j0 = c * tpr * VE + tc * VE;
                    VT w = row_ld<NTL>(reinterpret_cast<gptr<const VT>>(Wi + j0));
#pragma unroll
                    for (int e = 0; e < VE; ++e) {
                        const int j = j0 + e;
                        T cur = vget<VT, T>(w, e);
                        if (fix) cur = (j == cpp) ? yp : div_pivot(cur, pp, yp, pp_ok);
                        vset<VT, T>(w, e, update(cur, c, e, j));
                    }
                    row_st<NTL>(reinterpret_cast<gptr<VT>>(Wi + j0), w);
                }
            }
        }
    };
    // rows of a unit into wb: every slot, so that the memory counters stay
    // exact (slots without a row read the pivot row); in det_only mode only
    // the rows still needed, after the barrier that says which they are
    auto load_rows = [&](int i0, int nr, const int *srl, bool all) {
#pragma unroll
        for (int g = 0; g < B; ++g) {
            const int x = rsub + g * rg, i = i0 + x;
            const bool use = x < nr && i != rp;
            if (all || (use && srl[x] >= 0)) {
                const gptr<const T> Wi = W + (int64_t)(use ? i : rp) * ldw;
#pragma unroll
                for (int c = 0; c < NCH; ++c)
                    if (all || c < nch)
                        wb[g][c] = row_ld<NTL>(reinterpret_cast<gptr<const VT>>(Wi + (c < nch ? c : 0) * tpr * VE + tc * VE));
                if constexpr (RHS) wbb[g] = row_ld<NTL>(reinterpret_cast<gptr<const VT>>(Wi + bcol));
            }
        }
    };
    auto sweep_unit = [&](int i0, int nr, const T *sq, const int *srl) {
#pragma unroll
        for (int g = 0; g < B; ++g) {
            const int x = rsub + g * rg;
            if (x >= nr) continue;
            const int rn = srl[x];
            if (i0 + x == rp || rn < 0) continue;   // pivot row: written at step k+1
            sweep_row(g, i0 + x, sq[x], rn);
        }
    };

    if constexpr (!CNT) {   // own rows only
        if (kEarlyRows<NT> && !early) load_rows(r0, min(U, nsr), s_rls, false);
        for (int xg = 0; xg < nsr; xg += U) {
            sweep_unit(r0 + xg, min(U, nsr - xg), s_qs + xg, s_rls + xg);
            if (kEarlyRows<NT> && xg + U < nsr)
                load_rows(r0 + xg + U, min(U, nsr - xg - U), s_rls + xg + U, false);
        }
    } else {
    // The units in sweep order: the workgroup's own (positions 0 .. nstat-1,
    // multipliers already in LDS, no barrier), then units from the counter.
    // A counted unit's multipliers and indices pass through LDS together
    // with the id of the unit after it (the multiplier a_ik is overwritten
    // during the sweep by whichever thread holds that column, so it is read
    // before the barrier that precedes the sweep).  Thread 0 reads the
    // counter one unit before the id is published; the first read happens
    // during the second-to-last own unit, so the reads of different
    // workgroups are spread over the step and their latency is hidden.
    const gptr<int32_t> tick = &hdr->ticket[k & 1];
    int tk = 0;
    auto take = [&]() { tk = __hip_atomic_fetch_add(tick, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); };
    T qv = (T)0;
    int rov = 0;
    // the next unit's multiplier and old logical row index for thread t,
    // requested ahead of this unit's stores (nobody else writes its rows, and
    // the publishing barrier then does not wait for the stores)
    auto load_meta = [&](int uu) {
        const int i0 = uu * U + min(t, U - 1);
        const int i = (uu < nunits && i0 < n) ? i0 : rp;
        qv = W[(int64_t)i * ldw + cp];
        rov = rl_old[i];
    };
    auto publish = [&](int pr, int uu) {
        const int i = uu * U + t;
        if (t < U && i < n) row_meta(i, qv, rov, s_qd[pr], s_rld[pr], t);
        if (t == 0) {
            const int u2 = dyn0 + tk;
            s_nx[pr] = u2;
            if (u2 < nunits) take();
        }
    };
    const int tj = max(nstat - 2, 0);   // position during which the first counter read happens
    int u = nstat > 0 ? s0 : nunits, d1 = nunits, par = 1;
    const T *sq = s_qs;
    const int *srl = s_rls;
    for (int j = 0; u < nunits; ++j) {
        const bool next_counted = j + 1 >= nstat;
        int un = next_counted ? (j + 1 == nstat ? d1 : s_nx[par]) : s0 + j + 1;
        if (dyn) {
            if (t == 0 && j == tj) take();
            if (next_counted && !(nstat == 1 && j == 0)) load_meta(un);
        }
        const int nr = min(U, n - u * U);
        if (kEarlyRows<NT> && !early) load_rows(u * U, nr, srl, false);   // det_only: after its barrier
        sweep_unit(u * U, nr, sq, srl);
        if (dyn && j == tj) {   // publish the first counted unit's id
            if (t == 0) s_first = dyn0 + tk;
            __syncthreads();
            d1 = s_first;
            if (t == 0 && d1 < nunits) take();
            if (nstat == 1) { un = d1; load_meta(un); }
        }
        if (un >= nunits) break;
        if (early) load_rows(un * U, min(U, n - un * U), s_rls, true);
        if (!next_counted) {
            sq = s_qs + (j + 1) * U;
            srl = s_rls + (j + 1) * U;
        } else {
            par ^= 1;
            publish(par, un);
            __syncthreads();
            sq = s_qd[par];
            srl = s_rld[par];
        }
        u = un;
    }
    }
    if (k + 1 < n) {
        const int any_nf = __syncthreads_or(nf ? 1 : 0);
        // (the reductions compare |a|: RULE 2's "no candidate" score -1 goes
        // out as 0 with key 0xFFFFFFFF, below every real candidate)
        double bv = (double)bvT, ba = (RULE == 2) ? fmax((double)bsT, 0.0) : fabs(bv);
        block_argmax<NT>(ba, bv, bk, bi, bj, s_a, s_v, s_k, s_i, s_j);
        if (t == 0) {
            BigPart o;
            o.a = any_nf ? __builtin_inf() : ba;
            o.v = bv;
            o.rlog = (int32_t)(bk >> 16);
            o.clog = (int32_t)(bk & 0xFFFFu);
            o.iphys = bi;
            o.jphys = bj;
            glb(d.part)[(size_t)((k + 1) & 1) * d.nblk + rb] = o;
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
    // eq. 13: the product runs on one thread in step order; the records pass
    // through LDS in chunks, so that it does not wait on global memory at
    // every step
    if (bm.y == 0) {
        if (status == 0) {
            constexpr int kChunk = 1024;
            __shared__ T s_p[kChunk];
            __shared__ int s_flip[kChunk];
            DetAcc<T> det;
            det.init();
            for (int b0 = 0; b0 < n; b0 += kChunk) {
                const int cnt = min(kChunk, n - b0);
                for (int y = t; y < cnt; y += 256) {
                    const StepRec s = d.steps[b0 + y];
                    s_p[y] = (T)s.p;
                    s_flip[y] = (s.rlog != b0 + y) ^ (s.clog != b0 + y);
                }
                __syncthreads();
                if (t == 0)
                    for (int y = 0; y < cnt; ++y) {
                        det.mul(s_p[y]);
                        if (s_flip[y]) det.sign = -det.sign;
                    }
                __syncthreads();
            }
            if (t == 0) write_result_ok(d.res, n, det);
        } else if (t == 0) {
            write_result_fail(d.res, status, rank);
        }
    }
}

// X(i, j) = W(rowphys[collog[i]], colphys[rowlog[j]]), or for a solve
// X(i, j) = W(rowphys[collog[i]], n + j); the last pivot row still needs its
// eq. 14 division.  One workgroup per output row.
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
    const int m = d.ncol - d.rhs0;      // right-hand sides (0: inverse)
    const int ncx = m > 0 ? m : n;      // columns of X
    for (int i = bm.y; i < n; i += d.nblk) {
        double *Xi = d.X + (int64_t)i * d.ldx;
        if (status != 0) {
            for (int j = t; j < ncx; j += 256) Xi[j] = __builtin_nan("");
            continue;
        }
        const int src = d.rowphys[cl[i]];
        const T *Ws = W + (int64_t)src * d.ldw;
        const bool fix = (src == last.rphys);
        const T pl = (T)last.p;
        for (int j = t; j < ncx; j += 256) {
            const int sc = m > 0 ? d.rhs0 + j : d.colphys[rl[j]];
            T x = Ws[sc];
            if (fix) x = ((sc == last.cphys) ? one : x) / pl;
            Xi[j] = (double)x;
        }
    }
}

// ---------------------------------------------------------------- launchers

template <typename T, int NT, bool NTL, bool FULL, bool CNT, bool RHS = false, int RULE = 0,
          int NCH = kNch>
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
        hipLaunchKernelGGL((gj_big_step<T, NT, NTL, FULL, CNT, RHS, RULE, NCH>), dim3(grid_per_step ? grid_per_step[k] : grid_init),
                           dim3(NT), 0, s, descs, bmap, single, k, zero_tol, eps_default, det_only,
                           run_flag);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (events && events[1]) {
        e = hipEventRecord((hipEvent_t)events[1], s);
        if (e != hipSuccess) return e;
    }
    if (grid_finish == 0) return hipSuccess;   // steps only (a panel of the blocked elimination)
    hipLaunchKernelGGL((gj_big_finish<T>), dim3(grid_finish), dim3(256), 0, s, descs, bmap, single, run_flag);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!det_only && gather_grid > 0) {
        hipLaunchKernelGGL((gj_big_gather<T>), dim3(gather_grid), dim3(256), 0, s, descs, bmap, single, run_flag);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_big(bool fp32, int nt, bool nt_loads, int full, bool counted, bool rhs, int rule,
                      const BigDesc *descs, const int2 *bmap,
                      const BigDesc &single, const int *grid_per_step, int grid_init, int grid_finish, int max_n,
                      int gather_grid, double zero_tol, double eps_default, int det_only,
                      void *const *events, const int32_t *run_flag, hipStream_t s) {
    // full: 0 (per-chunk tests) or the chunk count 1-8 that every row fills
    // exactly (below 8: 256 and 512 threads, rule 0, no counter, no B).  The
    // counter is compiled in for 8 full chunks below 1024 threads only; the
    // extra right-hand-side chunk for FP64 with 8 full chunks below 1024
    // threads, without the counter
    if (full != 0 && (full < 1 || full > kNch)) return hipErrorInvalidValue;
    if (full != 0 && full != kNch && (counted || rhs || rule != 0 || nt >= 1024))
        return hipErrorInvalidValue;
    if (counted && !(full == kNch && nt < 1024)) return hipErrorInvalidValue;
    if (rhs && (fp32 || counted || full != kNch || nt >= 1024)) return hipErrorInvalidValue;
    // the other pivot rules: FP64, per-chunk tests, no counter, B right after A
    if (rule != 0 && (fp32 || counted || full || rhs || rule > 2)) return hipErrorInvalidValue;
#define GJ_BIG_ARGS descs, bmap, single, grid_per_step, grid_init, grid_finish, max_n, gather_grid, \
                    zero_tol, eps_default, det_only, events, run_flag, s
#define GJ_BIG_NCH(TT, NTV, C)                                                                    \
    case C:                                                                                       \
        return nt_loads ? run_big_t<TT, NTV, true, true, false, false, 0, C>(GJ_BIG_ARGS)         \
                        : run_big_t<TT, NTV, false, true, false, false, 0, C>(GJ_BIG_ARGS)
#define GJ_BIG_CASE(TT, NTV)                                                                      \
    if constexpr (!std::is_same<TT, float>::value) {                                              \
        if (rule == 1)                                                                            \
            return nt_loads ? run_big_t<TT, NTV, true, false, false, false, 1>(GJ_BIG_ARGS)       \
                            : run_big_t<TT, NTV, false, false, false, false, 1>(GJ_BIG_ARGS);     \
        if (rule == 2)                                                                            \
            return nt_loads ? run_big_t<TT, NTV, true, false, false, false, 2>(GJ_BIG_ARGS)       \
                            : run_big_t<TT, NTV, false, false, false, false, 2>(GJ_BIG_ARGS);     \
    }                                                                                             \
    if constexpr (NTV < 1024 && !std::is_same<TT, float>::value) {                                \
        if (rhs)                                                                                  \
            return nt_loads ? run_big_t<TT, NTV, true, true, false, true>(GJ_BIG_ARGS)            \
                            : run_big_t<TT, NTV, false, true, false, true>(GJ_BIG_ARGS);          \
    }                                                                                             \
    if constexpr (NTV < 1024) {                                                                   \
        if (counted)                                                                              \
            return nt_loads ? run_big_t<TT, NTV, true, true, true>(GJ_BIG_ARGS)                   \
                            : run_big_t<TT, NTV, false, true, true>(GJ_BIG_ARGS);                 \
        switch (full) {                                                                           \
            GJ_BIG_NCH(TT, NTV, 1); GJ_BIG_NCH(TT, NTV, 2); GJ_BIG_NCH(TT, NTV, 3);              \
            GJ_BIG_NCH(TT, NTV, 4);                                                               \
            GJ_BIG_NCH(TT, NTV, 5);                                                               \
            GJ_BIG_NCH(TT, NTV, 6); GJ_BIG_NCH(TT, NTV, 7);                                       \
            default: break;                                                                       \
        }                                                                                         \
    }                                                                                             \
    return nt_loads ? (full ? run_big_t<TT, NTV, true, true, false>(GJ_BIG_ARGS)                  \
                            : run_big_t<TT, NTV, true, false, false>(GJ_BIG_ARGS))                \
                    : (full ? run_big_t<TT, NTV, false, true, false>(GJ_BIG_ARGS)                 \
                            : run_big_t<TT, NTV, false, false, false>(GJ_BIG_ARGS))
    if (fp32) {
        switch (nt) {
            case 256: { GJ_BIG_CASE(float, 256); }
            case 512: { GJ_BIG_CASE(float, 512); }
            case 1024: { GJ_BIG_CASE(float, 1024); }
        }
    } else {
        switch (nt) {
            case 256: { GJ_BIG_CASE(double, 256); }
            case 512: { GJ_BIG_CASE(double, 512); }
            case 1024: { GJ_BIG_CASE(double, 1024); }
        }
    }
#undef GJ_BIG_CASE
#undef GJ_BIG_NCH
#undef GJ_BIG_ARGS
    return hipErrorInvalidValue;
}

size_t big_part_bytes() { return sizeof(BigPart); }
size_t big_step_bytes() { return sizeof(StepRec); }
size_t big_hdr_bytes() { return sizeof(BigHdr); }
size_t big_desc_bytes() { return sizeof(BigDesc); }

}  // namespace gj
