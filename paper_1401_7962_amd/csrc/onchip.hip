// onchip.hip -- full-pivot Gauss-Jordan with the matrix held in registers.
//
// One matrix per 256-thread workgroup (kind 0, a 16 x 16 thread grid) or per
// wavefront (kind 1, an 8 x 8 lane grid).  The n x n array (the in-place
// [A|D] of eqs. 3-10) is distributed cyclically: thread (tr, tc) holds rows
// a*TR + tr and columns b*TC + tc, E x E values in VGPRs, with E the smallest
// register block that covers n (n <= TR E), so padding costs at most
// (1 + 1/E)^2 of the real work.
//
// One step k (paper section 2):
//   1. the winner of the pivot search (Obs. 2-3) is already known from the
//      fused argmax of the previous step (largest |a| over the trailing block,
//      ties to the lowest row then column);
//   2. singular / non-finite test against the zero threshold (Obs. 2);
//   3. rows k,r and columns k,c are swapped physically: the owners of the four
//      lines stage them in LDS (the pivot row with slot k = 1, the pivot
//      column holding the multipliers a_ik), and every thread divides its own
//      entries of the pivot row by the pivot (eq. 14, correctly rounded, so
//      slot (k,k) becomes 1/p);
//   4. every element takes one fma with the staged row and column (eq. 15);
//      the pivot row is then overwritten with its scaled values;
//   5. while the new values are in registers, each thread scans its part of
//      the next trailing block in row-major order (so strict '>' keeps the
//      first maximum), and the workgroup reduces (|a|, row<<16|col).
// The determinant (eq. 13) is multiplied up in step order as an exact
// mantissa/exponent pair.  The final depivoting (Obs. 3) is folded into the
// store: element (i, j) of the working array goes to X(g[i], h[j]), where g
// (h) follows row i (column j) through the column (row) swaps of the result
// in reverse step order; one thread traces each index at the end.
#include <algorithm>

#include "gj_launch.h"

namespace gj {

template <typename T, int N, int NW>
struct CoreLds {
    // Positions >= n (padding) hold 0 in every array and in the registers: the
    // swap maps fix them, so padding lanes stage 0 onto 0, and a 0 never wins
    // the pivot search.  No per-element bounds test is needed.
    T prow[N + 1]; // new pivot row, not yet divided (slot k = 1); the pivot in slot N
    T pcol[N];     // new pivot column (multipliers)
    T newr[N];     // new row r  (= old row k, columns swapped)
    T newc[N];     // new column c (= old column k, rows swapped)
    int32_t g[N];  // destination row of working row i
    int32_t h[N];  // destination column of working column j
    int32_t ip[N]; // pivot sequence, written out once at the end (a global
    int32_t jp[N]; // store inside the step loop would make every barrier wait for it)
    T red_v[NW];   // each wavefront's largest |a| and its position key
    uint32_t red_k[NW];
};

template <int NW>
__device__ inline void group_sync() {
    if constexpr (NW > 1) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
}

// Largest of the 64 lanes' values, in every lane (values are |a| >= 0).
template <typename T, int CTRL>
__device__ inline T dpp_move(T x) {
    uint32_t w[Lanes<T>::W];
    Lanes<T>::split(x, w);
#pragma unroll
    for (int i = 0; i < Lanes<T>::W; ++i) w[i] = dpp_u32<CTRL>(w[i]);
    return Lanes<T>::join(w);
}

template <typename T>
__device__ inline T maxT(T a, T b) { return a > b ? a : b; }

template <typename T, bool P32>
__device__ inline T perm_max(T x) {
    uint32_t w[Lanes<T>::W], a[Lanes<T>::W], b[Lanes<T>::W];
    Lanes<T>::split(x, w);
#pragma unroll
    for (int i = 0; i < Lanes<T>::W; ++i) {
        auto p = P32 ? __builtin_amdgcn_permlane32_swap(w[i], w[i], false, false)
                     : __builtin_amdgcn_permlane16_swap(w[i], w[i], false, false);
        a[i] = p[0];
        b[i] = p[1];
    }
    return maxT(Lanes<T>::join(a), Lanes<T>::join(b));
}

template <typename T>
__device__ inline T wave_max(T m) {
    m = maxT(m, dpp_move<T, 0xB1>(m));    // quad_perm [1,0,3,2]
    m = maxT(m, dpp_move<T, 0x4E>(m));    // quad_perm [2,3,0,1]
    m = maxT(m, dpp_move<T, 0x141>(m));   // row_half_mirror
    m = maxT(m, dpp_move<T, 0x140>(m));   // row_mirror
    m = perm_max<T, false>(m);
    m = perm_max<T, true>(m);
    return m;
}

// Smallest of the 64 lanes' keys, in every lane.
__device__ inline uint32_t wave_min_u32(uint32_t x) {
    x = min(x, dpp_u32<0xB1>(x));
    x = min(x, dpp_u32<0x4E>(x));
    x = min(x, dpp_u32<0x141>(x));
    x = min(x, dpp_u32<0x140>(x));
    auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    x = min(p[0], p[1]);
    auto q = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return min(q[0], q[1]);
}

// Reduce (|a|, key) over the group: the largest value, ties to the smallest
// key (the first in row-major order).  The wavefront reduces the value
// alone; a ballot names the lanes that hold it, and only when several do
// are their keys reduced too.  The wavefronts' winners meet in LDS.  Every
// thread ends with the same winner.
template <typename T, int N, int NW>
__device__ inline void group_argmax(Cand<T> &c, CoreLds<T, N, NW> &L, int t) {
    const T m = wave_max(c.v);
    const bool have = (c.v == m) & (c.key != 0xFFFFFFFFu);
    const unsigned long long eq = __ballot(have);
    uint32_t key;
    if (eq == 0ull) {
        key = 0xFFFFFFFFu;                                  // nothing left to search
    } else if ((eq & (eq - 1ull)) == 0ull) {                // one lane holds the maximum
        key = (uint32_t)__builtin_amdgcn_readlane((int)c.key, __builtin_ctzll(eq));
    } else {                                                // equal maxima: the smallest key
        key = wave_min_u32(have ? c.key : 0xFFFFFFFFu);
    }
    if constexpr (NW > 1) {
        const int w = t / kWave;
        if ((t & (kWave - 1)) == 0) {
            L.red_v[w] = m;
            L.red_k[w] = key;
        }
        __syncthreads();
        T bv = L.red_v[0];
        uint32_t bk = L.red_k[0];
#pragma unroll
        for (int x = 1; x < NW; ++x) {
            const T ov = L.red_v[x];
            const uint32_t ok = L.red_k[x];
            const bool take = (ov > bv) | ((ov == bv) & (ok < bk));
            bv = take ? ov : bv;
            bk = take ? ok : bk;
        }
        c.v = bv;
        c.key = bk;
    } else {
        c.v = m;
        c.key = key;
    }
}

// Scan this thread's part of the trailing block (rows and columns > k) in
// row-major order; strict '>' keeps the first maximum (padding holds 0 and
// never wins).  Register rows whose rows are all pivoted are skipped (a
// wavefront-uniform branch); within a row the pivoted columns are masked per
// lane, which costs less than a branch per element.  The candidate
// carries |a| and the position; the owners of the winning row recover the
// signed pivot when they stage it.  The winning slot is tracked as the
// compile-time code a*EB+b, so no per-element key stays live across steps,
// and the lane masks are combined with '&' (no short-circuit branches).
template <typename T, int TR, int TC, int EA, int EB>
__device__ __forceinline__ void scan_argmax(const T (&v)[EA][EB], int k, int tr, int tc,
                                            Cand<T> &c) {
    using M = Num<T>;
    bool cok[EB];
#pragma unroll
    for (int b = 0; b < EB; ++b) cok[b] = (b * TC + tc > k);
    // two running maxima (even and odd register rows: independent chains)
    constexpr int NCH = EA < 2 ? EA : 2;
    T rbest[NCH];
    int rcode[NCH];
#pragma unroll
    for (int h = 0; h < NCH; ++h) { rbest[h] = (T)0; rcode[h] = -1; }
#pragma unroll
    for (int a = 0; a < EA; ++a) {
        if (a * TR + TR - 1 <= k) continue;        // every row of this block pivoted
        const bool rok = (a * TR + tr > k);
        const int h = a % NCH;
#pragma unroll
        for (int b = 0; b < EB; ++b) {
            const T ax = M::abs_(v[a][b]);
            const bool gt = rok & cok[b] & (ax > rbest[h]);
            rbest[h] = gt ? ax : rbest[h];
            rcode[h] = gt ? (a * EB + b) : rcode[h];
        }
    }
    // merge the chains: on equal values the smaller slot code (earlier in
    // row-major order) wins
    T best = rbest[0];
    int code = rcode[0];
#pragma unroll
    for (int h = 1; h < NCH; ++h) {
        const bool gt = (rbest[h] > best) | ((rbest[h] == best) & (rcode[h] >= 0) &
                                               ((unsigned)rcode[h] < (unsigned)code));
        best = gt ? rbest[h] : best;
        code = gt ? rcode[h] : code;
    }
    c.v = best;
    const int i = (code / EB) * TR + tr, j = (code % EB) * TC + tc;
    c.key = (code >= 0) ? (((uint32_t)i << 16) | (uint32_t)j) : 0xFFFFFFFFu;
}

// STATIC: the pivot of step k is element (k, k) (the rows and columns are
// already in pivot order, as for the refined path's determinant blocks); no
// search, and the singular test looks at that element.
template <typename T, int TR, int TC, int EA, int EB, int NW, bool STATIC = false>
__device__ __forceinline__ void gj_core(int t, const MatDesc md, const double *__restrict__ A,
                                        double *__restrict__ X, int32_t *__restrict__ ipiv_all,
                                        int32_t *__restrict__ jpiv_all,
                                        gj_result *__restrict__ res_all, double zero_tol,
                                        double eps_default, int det_only,
                                        CoreLds<T, TR * EA, NW> &L) {
    constexpr int N = TR * EA;
    static_assert(TR * EA == TC * EB, "square tiling");
    static_assert(TR * TC == NW * kWave, "thread grid");
    using M = Num<T>;
    if (md.run && *md.run == 0) return;   // same test in every thread of the group
    const int n = md.n;
    const int tr = t / TC, tc = t % TC;
    int32_t *ipiv = ipiv_all + md.piv_off;
    int32_t *jpiv = jpiv_all + md.piv_off;
    gj_result *res = res_all + md.res_idx;

    T v[EA][EB];
    bool bad = false;
#pragma unroll
    for (int a = 0; a < EA; ++a) {
        const int i = a * TR + tr;
#pragma unroll
        for (int b = 0; b < EB; ++b) {
            const int j = b * TC + tc;
            v[a][b] = (i < n && j < n) ? (T)A[md.a_off + (int64_t)i * md.lda + j] : (T)0;
            bad |= !M::finite_(v[a][b]);
        }
    }
    for (int x = t; x < N; x += TR * TC) {
        L.prow[x] = (T)0;
        L.pcol[x] = (T)0;
        L.newr[x] = (T)0;
        L.newc[x] = (T)0;
    }

    // Non-finite candidates: every candidate of step 0 is checked here.  After
    // that only an overflow to +-inf can make a candidate non-finite (with
    // full pivoting |a_kj / p| <= 1 on the candidate columns, so no 0 * inf
    // arises), and an infinity always wins the pivot search; so testing the
    // winner is enough for the later steps.
    Cand<T> c;
    scan_argmax<T, TR, TC, EA, EB>(v, -1, tr, tc, c);
    group_argmax(c, L, t);
    bool nf;
    if constexpr (NW == 1) {
        nf = __any(bad ? 1 : 0) != 0;
    } else {
        nf = __syncthreads_or(bad ? 1 : 0) != 0;
    }

    const T tau = (zero_tol >= 0.0) ? (T)zero_tol : (T)n * (T)eps_default * M::abs_(c.v);
    DetAcc<T> det;
    det.init();
    int code = GJ_RES_OK, rank = n;

    for (int k = 0; k < n; ++k) {
        if constexpr (!STATIC) {
            const T m = c.v;   // |pivot|
            if (nf || !M::finite_(m)) { code = GJ_RES_NONFINITE; rank = k; break; }
            if (m == (T)0 || m < tau) { code = GJ_RES_SINGULAR; rank = k; break; }
        }
        const int r = STATIC ? k : (int)(c.key >> 16), cc = STATIC ? k : (int)(c.key & 0xFFFFu);
        const int ar = r / TR, trr = r % TR, ak = k / TR, trk = k % TR;
        const int bc = cc / TC, tcc = cc % TC, bk = k / TC, tck = k % TC;

        // Stage the four swapped lines in LDS.  Each entry goes straight to
        // its slot after the swaps (rows r,k and columns c,k exchanged): the
        // slots form a permutation, so no slot is written by two wavefronts
        // and the readers need no fix-ups.  Row r goes out unscaled; its
        // pivot goes to slot N and its pivot slot (column k after the swap)
        // is set to 1, so that after the barrier every thread divides its own
        // entries by the pivot (eq. 14) and 1/p, the pivot slot of D, comes
        // out of the same correctly rounded division.  (Dividing here, in the
        // one wavefront that owns row r, would keep the others waiting.)
        const bool lane_r = (tr == trr), lane_k = (tr == trk);
        const bool lane_c = (tc == tcc), lane_ck = (tc == tck);
        if (lane_r) {
#pragma unroll
            for (int a = 0; a < EA; ++a)
                if (a == ar) {
#pragma unroll
                    for (int b = 0; b < EB; ++b) {
                        int j = b * TC + tc;
                        j = (lane_ck & (b == bk)) ? cc : j;
                        j = (lane_c & (b == bc)) ? N : j;
                        L.prow[j] = v[a][b];
                    }
                    if (lane_c) L.prow[k] = M::one();   // after the write above, same lane
                }
        }
        if (lane_k) {                          // old row k -> row r, columns swapped
#pragma unroll
            for (int a = 0; a < EA; ++a)
                if (a == ak) {
#pragma unroll
                    for (int b = 0; b < EB; ++b) {
                        int j = b * TC + tc;
                        j = (lane_ck & (b == bk)) ? cc : j;
                        j = (lane_c & (b == bc)) ? k : j;
                        L.newr[j] = v[a][b];
                    }
                }
        }
        if (lane_c | lane_ck) {
            int ri[EA];                        // slot of each register row after the row swap
#pragma unroll
            for (int a = 0; a < EA; ++a) {
                int i = a * TR + tr;
                i = (lane_k & (a == ak)) ? r : i;
                i = (lane_r & (a == ar)) ? k : i;
                ri[a] = i;
            }
            if (lane_c) {                      // the multipliers
#pragma unroll
                for (int b = 0; b < EB; ++b)
                    if (b == bc) {
#pragma unroll
                        for (int a = 0; a < EA; ++a) L.pcol[ri[a]] = v[a][b];
                    }
            }
            if (lane_ck) {                     // old column k -> column c
#pragma unroll
                for (int b = 0; b < EB; ++b)
                    if (b == bk) {
#pragma unroll
                        for (int a = 0; a < EA; ++a) L.newc[ri[a]] = v[a][b];
                    }
            }
        }
        if (t == 0) {
            L.ip[k] = r;
            L.jp[k] = cc;
        }
        group_sync<NW>();

        // eq. 13, in step order (every lane keeps the same product)
        const T p = L.prow[N];
        if constexpr (STATIC) {   // the same staged value in every thread
            const T ap = M::abs_(p);
            if (nf || !M::finite_(ap)) { code = GJ_RES_NONFINITE; rank = k; break; }
            if (ap == (T)0 || ap < tau) { code = GJ_RES_SINGULAR; rank = k; break; }
        }
        det.mul(p);
        if (r != k) det.sign = -det.sign;
        if (cc != k) det.sign = -det.sign;

        // install the swapped row r and column c; clear column k (it becomes
        // fma(-q, 1/p, 0) below, the D column of eq. 15; when c = k the clear
        // comes last)
        if (lane_r) {
#pragma unroll
            for (int a = 0; a < EA; ++a)
                if (a == ar) {
#pragma unroll
                    for (int b = 0; b < EB; ++b) v[a][b] = L.newr[b * TC + tc];
                }
        }
        if (lane_c) {
#pragma unroll
            for (int b = 0; b < EB; ++b)
                if (b == bc) {
#pragma unroll
                    for (int a = 0; a < EA; ++a) v[a][b] = L.newc[a * TR + tr];
                }
        }
        if (lane_ck) {
#pragma unroll
            for (int b = 0; b < EB; ++b)
                if (b == bk) {
#pragma unroll
                    for (int a = 0; a < EA; ++a) v[a][b] = (T)0;
                }
        }
        // eq. 14 on this thread's columns of the pivot row; eq. 15 for every
        // row, then the pivot row takes its scaled values
        const T y = M::one() / p;
        const bool p_ok = div_pivot_ok(p);
        T q[EA], pr[EB], xr[EB];
#pragma unroll
        for (int b = 0; b < EB; ++b) xr[b] = L.prow[b * TC + tc];
#pragma unroll
        for (int a = 0; a < EA; ++a) q[a] = L.pcol[a * TR + tr];
        bool slow = false;
#pragma unroll
        for (int b = 0; b < EB; ++b) pr[b] = div_pivot_fast(xr[b], p, y, p_ok, slow);
        if (slow) {   // operands outside the corrected-quotient range
#pragma unroll
            for (int b = 0; b < EB; ++b) pr[b] = div_pivot(xr[b], p, y, p_ok);
        }
#pragma unroll
        for (int a = 0; a < EA; ++a)
#pragma unroll
            for (int b = 0; b < EB; ++b) v[a][b] = M::fma_(-q[a], pr[b], v[a][b]);
        if (tr == trk) {
#pragma unroll
            for (int a = 0; a < EA; ++a)
                if (a == ak) {
#pragma unroll
                    for (int b = 0; b < EB; ++b) v[a][b] = pr[b];
                }
        }
        // fused pivot search for step k+1 over rows and columns > k (with
        // static pivots only the barrier that keeps the next step's staging
        // from overwriting lines another wavefront still reads)
        if (k + 1 < n) {
            if constexpr (STATIC) {
                group_sync<NW>();
            } else {
                scan_argmax<T, TR, TC, EA, EB>(v, k, tr, tc, c);
                group_argmax(c, L, t);
            }
        }
    }

    // Depivoting maps: g (h) follows working row i (column j) through the
    // column (row) swaps of the result, undone in reverse step order; one
    // thread per index.
    group_sync<NW>();
    for (int x = t; x < 2 * N; x += TR * TC) {
        const bool row = x < N;
        const int i0 = row ? x : x - N;
        int pos = i0;
        if (code == GJ_RES_OK && i0 < n) {
            const int32_t *sw = row ? L.jp : L.ip;
            for (int kk = n - 1; kk >= 0; --kk) {
                const int s2 = sw[kk];
                pos = (pos == kk) ? s2 : ((pos == s2) ? kk : pos);
            }
        }
        if (row) L.g[i0] = pos; else L.h[i0] = pos;
    }
    group_sync<NW>();
    for (int x = t; x < n; x += TR * TC) {
        ipiv[x] = (x < rank) ? L.ip[x] : -1;
        jpiv[x] = (x < rank) ? L.jp[x] : -1;
    }
    if (code == GJ_RES_OK) {
        if (!det_only) {
#pragma unroll
            for (int a = 0; a < EA; ++a) {
                const int i = a * TR + tr;
                if (i < n) {
                    const int64_t row = md.x_off + (int64_t)L.g[i] * md.ldx;
#pragma unroll
                    for (int b = 0; b < EB; ++b) {
                        const int j = b * TC + tc;
                        if (j < n) X[row + L.h[j]] = (double)v[a][b];
                    }
                }
            }
        }
        if (t == 0) write_result_ok(res, n, det);
    } else {
        if (!det_only) {
            const double qnan = __builtin_nan("");
            for (int a = 0; a < EA; ++a) {
                const int i = a * TR + tr;
                if (i < n)
                    for (int b = 0; b < EB; ++b) {
                        const int j = b * TC + tc;
                        if (j < n) X[md.x_off + (int64_t)i * md.ldx + j] = qnan;
                    }
            }
        }
        if (t == 0) write_result_fail(res, code, rank);
    }
}

// Persistent kernel for one class of tasks: KIND 0 = one matrix on all four
// wavefronts (16 x 16 threads, E x E values each, n <= 16 E); KIND 1 = one
// matrix per wavefront (8 x 8 lanes, n <= 8 E).  Workgroups take tasks from
// an atomic queue until it is empty; tasks are ordered by decreasing cost on
// the host.  With mats == nullptr the kernel inverts the single matrix passed
// by value (workgroup 0, KIND 0).
// At least two wavefronts per SIMD: the register budget stays within 256.
template <typename T, int KIND, int E, bool STATIC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
gj_onchip_kernel(const MatDesc *__restrict__ mats, const OnchipTask *__restrict__ tasks,
                 int ntasks, uint32_t *__restrict__ queue, const MatDesc single,
                 const double *__restrict__ A, double *__restrict__ X, int32_t *__restrict__ ipiv,
                 int32_t *__restrict__ jpiv, gj_result *__restrict__ res, double zero_tol,
                 double eps_default, int det_only, const int32_t *__restrict__ run_flag) {
    using L0 = CoreLds<T, 16 * E, 4>;
    using L1 = CoreLds<T, 8 * E, 1>;
    constexpr size_t kBytes = KIND == 0 ? sizeof(L0) : 4 * sizeof(L1);
    __shared__ __attribute__((aligned(16))) unsigned char smem[kBytes];
    __shared__ int s_task;
    const int t = threadIdx.x;
    if (run_flag && *run_flag == 0) return;
    if (mats == nullptr) {
        if constexpr (KIND == 0) {
            if (blockIdx.x == 0)
                gj_core<T, 16, 16, E, E, 4, STATIC>(t, single, A, X, ipiv, jpiv, res, zero_tol,
                                            eps_default, det_only, *reinterpret_cast<L0 *>(smem));
        }
        return;
    }
    for (;;) {
        if (t == 0) s_task = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int id = s_task;
        __syncthreads();
        if (id >= ntasks) break;
        const OnchipTask task = tasks[id];
        if constexpr (KIND == 0) {
            const MatDesc md = mats[task.m[0]];
            gj_core<T, 16, 16, E, E, 4, STATIC>(t, md, A, X, ipiv, jpiv, res, zero_tol, eps_default,
                                        det_only, *reinterpret_cast<L0 *>(smem));
        } else {
            const int w = t / kWave, lane = t % kWave;
            const int mi = task.m[w];
            if (mi >= 0) {
                const MatDesc md = mats[mi];
                gj_core<T, 8, 8, E, E, 1, STATIC>(lane, md, A, X, ipiv, jpiv, res, zero_tol, eps_default,
                                          det_only, reinterpret_cast<L1 *>(smem)[w]);
            }
        }
        __syncthreads();
    }
}

__global__ void gj_zero_u32_kernel(uint32_t *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

// ---------------------------------------------------------------- launchers

hipError_t launch_zero_u32(uint32_t *p, int count, hipStream_t s) {
    hipLaunchKernelGGL(gj_zero_u32_kernel, dim3((count + 255) / 256), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

// Task classes: c = 0..7 is kind 0 with E = 8 - c (one matrix per workgroup,
// n <= 16 E), c = 8..15 is kind 1 with E = 16 - c (one matrix per
// wavefront, n <= 8 E).  A batch sends n > 64 to kind 0 and n <= 64 to kind
// 1, each with the smallest E that covers n, so the padded work stays below
// (1 + 1/E)^2 of the real work; classes run largest E first.  A single
// matrix always uses kind 0 (all four wavefronts).
int onchip_class_of(int n, bool single) {
    if (n < 1 || n > 128) return -1;
    if (single || n > 64) return 8 - (n + 15) / 16;
    return 16 - (n + 7) / 8;
}
int onchip_class_kind(int c) { return c < 8 ? 0 : 1; }

template <typename T, int KIND, int E, bool STATIC>
static hipError_t launch_cls(const MatDesc *mats, const OnchipTask *tasks, int ntasks,
                             uint32_t *queue, const MatDesc &single, int grid, const double *A,
                             double *X, int32_t *ipiv, int32_t *jpiv, gj_result *res,
                             double zero_tol, double eps_default, int det_only,
                             const int32_t *run_flag, hipStream_t s) {
    if (mats) {
        int dev = 0, cus = 256, per = 1;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gj_onchip_kernel<T, KIND, E, STATIC>, 256, 0) != hipSuccess) per = 1;
        const int force = env_int("GJ_ONCHIP_PER_CU", 0);   // experiments only
        if (force > 0) per = force;
        grid = std::max(1, std::min(ntasks, cus * std::max(per, 1)));
    }
    hipLaunchKernelGGL((gj_onchip_kernel<T, KIND, E, STATIC>), dim3(grid), dim3(256), 0, s, mats, tasks,
                       ntasks, queue, single, A, X, ipiv, jpiv, res, zero_tol, eps_default, det_only,
                       run_flag);
    return hipGetLastError();
}

template <typename T, bool STATIC>
static hipError_t launch_cls_t(int cls, const MatDesc *mats, const OnchipTask *tasks, int ntasks,
                               uint32_t *queue, const MatDesc &single, const double *A, double *X,
                               int32_t *ipiv, int32_t *jpiv, gj_result *res, double zero_tol,
                               double eps_default, int det_only, const int32_t *run_flag,
                               hipStream_t s) {
#define GJ_CLS(C, K, EE)                                                                        \
    case C:                                                                                     \
        return launch_cls<T, K, EE, STATIC>(mats, tasks, ntasks, queue, single, 1, A, X, ipiv,  \
                                            jpiv, res, zero_tol, eps_default, det_only,         \
                                            run_flag, s)
    switch (cls) {
        GJ_CLS(0, 0, 8); GJ_CLS(1, 0, 7); GJ_CLS(2, 0, 6); GJ_CLS(3, 0, 5);
        GJ_CLS(4, 0, 4); GJ_CLS(5, 0, 3); GJ_CLS(6, 0, 2); GJ_CLS(7, 0, 1);
        GJ_CLS(8, 1, 8); GJ_CLS(9, 1, 7); GJ_CLS(10, 1, 6); GJ_CLS(11, 1, 5);
        GJ_CLS(12, 1, 4); GJ_CLS(13, 1, 3); GJ_CLS(14, 1, 2); GJ_CLS(15, 1, 1);
    }
#undef GJ_CLS
    return hipErrorInvalidValue;
}

hipError_t launch_onchip_class(bool fp32, int cls, const MatDesc *mats, const OnchipTask *tasks,
                               int ntasks, uint32_t *queue, const MatDesc &single, const double *A,
                               double *X, int32_t *ipiv, int32_t *jpiv, gj_result *res,
                               double zero_tol, double eps_default, int det_only,
                               const int32_t *run_flag, hipStream_t s) {
    const bool stat = (det_only & kOnchipStaticPivots) != 0;   // FP64 only
    det_only &= 1;
    if (stat)
        return fp32 ? hipErrorInvalidValue
                    : launch_cls_t<double, true>(cls, mats, tasks, ntasks, queue, single, A, X, ipiv,
                                                 jpiv, res, zero_tol, eps_default, det_only, run_flag, s);
    return fp32 ? launch_cls_t<float, false>(cls, mats, tasks, ntasks, queue, single, A, X, ipiv, jpiv,
                                             res, zero_tol, eps_default, det_only, run_flag, s)
                : launch_cls_t<double, false>(cls, mats, tasks, ntasks, queue, single, A, X, ipiv, jpiv,
                                              res, zero_tol, eps_default, det_only, run_flag, s);
}

// Single matrix (n <= 128) on one workgroup.
hipError_t launch_onchip(bool fp32, const MatDesc *mats, const OnchipTask *tasks, int ntasks,
                         uint32_t *queue, const MatDesc &single, int grid, const double *A,
                         double *X, int32_t *ipiv, int32_t *jpiv, gj_result *res, double zero_tol,
                         double eps_default, int det_only, const int32_t *run_flag,
                         hipStream_t s) {
    (void)mats; (void)tasks; (void)ntasks; (void)queue; (void)grid;
    return launch_onchip_class(fp32, onchip_class_of(single.n, true), nullptr, nullptr, 0, nullptr,
                               single, A, X, ipiv, jpiv, res, zero_tol, eps_default, det_only,
                               run_flag, s);
}

}  // namespace gj
