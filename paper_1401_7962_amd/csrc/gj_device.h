// gj_device.h -- device-side types and helpers shared by the libgj kernels.
//
// Everything here is part of the product library (HIP, gfx950).  Numeric
// conventions (paper section 2):
//   * eq. 14 (pivot row / pivot) is a correctly rounded division;
//   * eq. 15 (row i minus a_ik times the new pivot row) is one fma per
//     element: w = fma(-q, prow_j, w);
//   * the pivot search (Obs. 2-3) takes the largest |a| of the trailing block;
//     ties go to the lowest row, then the lowest column, of the current
//     matrix;
//   * eq. 13's product of pivots is kept as (mantissa, exponent) with frexp
//     renormalisation after every multiplication.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gj.h"

namespace gj {

constexpr int kWave = 64;

template <typename T> struct Num;

template <> struct Num<double> {
    __device__ static inline double fma_(double a, double b, double c) { return fma(a, b, c); }
    __device__ static inline double abs_(double a) { return fabs(a); }
    __device__ static inline double frexp_(double a, int *e) { return frexp(a, e); }
    __device__ static inline bool finite_(double a) { return fabs(a) <= 1.7976931348623157e308; }
    __device__ static inline double one() { return 1.0; }
};

template <> struct Num<float> {
    __device__ static inline float fma_(float a, float b, float c) { return fmaf(a, b, c); }
    __device__ static inline float abs_(float a) { return fabsf(a); }
    __device__ static inline float frexp_(float a, int *e) { return frexpf(a, e); }
    __device__ static inline bool finite_(float a) { return fabsf(a) <= 3.40282346638528859812e+38f; }
    __device__ static inline float one() { return 1.0f; }
};

// x / p correctly rounded (eq. 14), from y = RN(1/p) computed once per step.
// Markstein's theorem: with y = RN(1/p) and q = RN(x y), the residual
// r = x - p q is exact (one fma) and RN(q + r y) = RN(x / p), provided no
// intermediate overflows or underflows.  That holds when x and p are normal
// with |exponent| <= 500 (FP64) or 60 (FP32); zeros give q exactly; any
// other operand takes the IEEE division.  (Checked against IEEE division on
// 4e8 random and all-ones-mantissa operand pairs per precision.)
template <typename T> struct DivRange;
template <> struct DivRange<double> {
    __device__ static constexpr double lo() { return 0x1p-500; }
    __device__ static constexpr double hi() { return 0x1p+500; }
};
template <> struct DivRange<float> {
    __device__ static constexpr float lo() { return 0x1p-60f; }
    __device__ static constexpr float hi() { return 0x1p+60f; }
};

template <typename T>
__device__ inline bool div_pivot_ok(T p) {
    const T ap = Num<T>::abs_(p);
    return ap >= DivRange<T>::lo() && ap <= DivRange<T>::hi();
}

// Straight-line part of div_pivot: the corrected quotient, and `slow` set
// when x lies outside the range where the correction is exact (the caller
// then redoes those elements with div_pivot, off the common path).
template <typename T>
__device__ __forceinline__ T div_pivot_fast(T x, T p, T y, bool p_ok, bool &slow) {
    const T ax = Num<T>::abs_(x);
    const T q = x * y;
    const T r = Num<T>::fma_(-p, q, x);
    const T res = (ax == (T)0) ? q : Num<T>::fma_(r, y, q);
    // bitwise operators: no short-circuit branches on the common path
    slow |= ((int)(ax == (T)0) | ((int)p_ok & (int)(ax >= DivRange<T>::lo()) &
                                  (int)(ax <= DivRange<T>::hi()))) == 0;
    return res;
}

template <typename T>
__device__ inline T div_pivot(T x, T p, T y, bool p_ok) {
    const T ax = Num<T>::abs_(x);
    const T q = x * y;
    const T r = Num<T>::fma_(-p, q, x);
    T res = (ax == (T)0) ? q : Num<T>::fma_(r, y, q);
    const bool fast = (ax == (T)0) || (p_ok && ax >= DivRange<T>::lo() && ax <= DivRange<T>::hi());
    if (!fast) res = x / p;
    return res;
}

// Running product of pivots (eq. 13) as mantissa * 2^exp, renormalised after
// every multiplication so that it neither overflows nor underflows.
template <typename T> struct DetAcc {
    T m;
    int64_t e;
    int sign;  // (-1)^(number of non-trivial swaps)
    __device__ inline void init() { m = Num<T>::one(); e = 0; sign = 1; }
    __device__ inline void mul(T p) {
        int e1, e2;
        T f = Num<T>::frexp_(p, &e1);
        m = m * f;
        e += e1;
        m = Num<T>::frexp_(m, &e2);
        e += e2;
    }
};

__device__ inline double ldexp64(double m, int64_t e) {
    if (e > 4000) e = 4000;
    if (e < -4000) e = -4000;
    return ldexp(m, (int)e);
}

template <typename T>
__device__ inline void write_result_ok(gj_result *res, int n, const DetAcc<T> &d) {
    res->code = GJ_RES_OK;
    res->rank = n;
    double mant = (double)d.m;
    res->det_sign = (mant < 0.0) ? -d.sign : d.sign;
    res->det_mant = fabs(mant);
    res->det_exp = d.e;
    res->det = ldexp64((double)d.sign * mant, d.e);
    res->logabsdet = log(fabs(mant)) + (double)d.e * 0.69314718055994530942;
    res->refine_iters = 0;
    res->resid = __builtin_nan("");
}

__device__ inline void write_result_fail(gj_result *res, int code, int rank) {
    res->code = code;
    res->rank = rank;
    res->det_sign = 0;
    res->det_mant = 0.0;
    res->det_exp = 0;
    if (code == GJ_RES_SINGULAR) {
        res->det = 0.0;
        res->logabsdet = -__builtin_inf();
    } else {
        res->det = __builtin_nan("");
        res->logabsdet = __builtin_nan("");
    }
    res->refine_iters = 0;
    res->resid = __builtin_nan("");
}

// Argmax candidate: largest |v|, ties to the smallest key.  key packs
// (row << 16 | col) of the current matrix, so unsigned order is row-major
// order.  "No candidate" is (0, 0xFFFFFFFF): it loses every comparison with a
// real candidate, zeros included.
template <typename T> struct Cand {
    T v;           // signed value
    uint32_t key;
};

template <typename T>
__device__ inline bool better(T v1, uint32_t k1, T v2, uint32_t k2) {
    const T a1 = Num<T>::abs_(v1), a2 = Num<T>::abs_(v2);
    return (a1 > a2) || (a1 == a2 && k1 < k2);
}

// ---- cross-lane moves without LDS: DPP within rows of 16 lanes, permlane
// swaps across rows (gfx950)
template <int CTRL>
__device__ inline uint32_t dpp_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xF, 0xF, false);
}

template <typename T> struct Lanes;
template <> struct Lanes<double> {
    static constexpr int W = 2;
    __device__ static inline void split(double v, uint32_t *w) {
        w[0] = (uint32_t)__double2loint(v);
        w[1] = (uint32_t)__double2hiint(v);
    }
    __device__ static inline double join(const uint32_t *w) {
        return __hiloint2double((int)w[1], (int)w[0]);
    }
};
template <> struct Lanes<float> {
    static constexpr int W = 1;
    __device__ static inline void split(float v, uint32_t *w) { w[0] = __float_as_uint(v); }
    __device__ static inline float join(const uint32_t *w) { return __uint_as_float(w[0]); }
};

template <typename T>
__device__ inline void cand_take(Cand<T> &c, T ov, uint32_t ok) {
    if (better(ov, ok, c.v, c.key)) { c.v = ov; c.key = ok; }
}

template <typename T, int CTRL>
__device__ inline void argmax_dpp_step(Cand<T> &c) {
    uint32_t w[Lanes<T>::W];
    Lanes<T>::split(c.v, w);
#pragma unroll
    for (int x = 0; x < Lanes<T>::W; ++x) w[x] = dpp_u32<CTRL>(w[x]);
    const uint32_t ok = dpp_u32<CTRL>(c.key);
    cand_take(c, Lanes<T>::join(w), ok);
}

// permlane{16,32}_swap with the same register as both operands leaves the
// pair (own row/half, partner row/half) in identical order in every lane of
// the pair, so combining the two halves gives every lane the same winner.
template <typename T, bool P32>
__device__ inline void argmax_perm_step(Cand<T> &c) {
    uint32_t w[Lanes<T>::W], a[Lanes<T>::W], b[Lanes<T>::W];
    Lanes<T>::split(c.v, w);
#pragma unroll
    for (int x = 0; x < Lanes<T>::W; ++x) {
        auto p = P32 ? __builtin_amdgcn_permlane32_swap(w[x], w[x], false, false)
                     : __builtin_amdgcn_permlane16_swap(w[x], w[x], false, false);
        a[x] = p[0];
        b[x] = p[1];
    }
    auto pk = P32 ? __builtin_amdgcn_permlane32_swap(c.key, c.key, false, false)
                  : __builtin_amdgcn_permlane16_swap(c.key, c.key, false, false);
    Cand<T> r;
    r.v = Lanes<T>::join(a);
    r.key = pk[0];
    cand_take(r, Lanes<T>::join(b), pk[1]);
    c = r;
}

// Every lane of the wavefront ends with the wavefront's winner.
template <typename T>
__device__ inline void wave_argmax(Cand<T> &c) {
    argmax_dpp_step<T, 0xB1>(c);   // quad_perm [1,0,3,2]
    argmax_dpp_step<T, 0x4E>(c);   // quad_perm [2,3,0,1]
    argmax_dpp_step<T, 0x141>(c);  // row_half_mirror
    argmax_dpp_step<T, 0x140>(c);  // row_mirror
    argmax_perm_step<T, false>(c);
    argmax_perm_step<T, true>(c);
}

// Descriptor of one matrix of a batch (offsets in elements).
struct MatDesc {
    int64_t a_off;
    int64_t x_off;
    int64_t piv_off;
    int32_t n;
    int32_t lda;
    int32_t ldx;
    int32_t res_idx;
    const int32_t *run;  // null, or a per-matrix flag: skip the matrix when 0
};

// On-chip task: kind 0 = one matrix on the whole 256-thread workgroup;
// kind 1 = up to four matrices, one per wavefront (m[w] < 0: none).
struct OnchipTask {
    int32_t kind;
    int32_t m[4];
};

// ---- streaming (large-n) path bookkeeping, one set per matrix
struct BigPart {          // one workgroup's candidate for the next pivot
    double a;             // |value|; +inf when a non-finite candidate was seen
    double v;             // signed value
    int32_t rlog, clog;   // logical (swapped) position
    int32_t iphys, jphys; // physical position in W
};

struct StepRec {          // what step k chose
    double p;
    int32_t rphys, cphys, rlog, clog;
};

struct BigHdr {
    int32_t status;       // 0 while running, else GJ_RES_* that stopped it
    int32_t rank;
    double tau;
    int32_t ticket[2];    // work-unit counters of the step kernel, by step parity
};

// Global-address-space views of device pointers.  Pointers read from a
// descriptor are generic to the compiler, which then emits FLAT accesses; a
// FLAT load counts against the LDS counter too, so every LDS wait would also
// wait for it.  Accesses through these views compile to global_load/store.
// (The host pass only type-checks kernel bodies; it sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T> using gptr = __attribute__((address_space(1))) T *;
#else
template <typename T> using gptr = T *;
#endif
template <typename T> __device__ __forceinline__ gptr<T> glb(T *p) { return (gptr<T>)p; }

struct BigDesc {
    void *W;              // T[n x ldw]
    int64_t ldw;
    BigPart *part;        // [2][nblk]
    int32_t *rowlog;      // [2][n] physical row -> logical row
    int32_t *collog;      // [2][n] physical column -> logical column
    int32_t *rowphys;     // [n] logical -> physical (filled at the end)
    int32_t *colphys;     // [n]
    StepRec *steps;       // [n]
    BigHdr *hdr;
    const double *A;
    int64_t lda;
    double *X;
    int64_t ldx;
    int32_t *ipiv, *jpiv;
    gj_result *res;
    int64_t mstride;      // stride between the two parities of a map (= ldw)
    const int32_t *run;   // null, or a per-matrix flag: every kernel skips it when 0
    int32_t n, R, nblk, tpr;  // order, rows per workgroup, workgroups, threads per row
    int32_t ustat;            // work units each workgroup of the step kernel takes statically
    int32_t ncol;             // columns of W in use: n, or rhs0 + m when solving for m right-hand sides
    int32_t rhs0;             // column of W holding B's first column (n when not solving)
    int32_t rule;             // pivot rule: 0 full (Obs. 2-3), 1 partial on |a|, 2 the program's (section 3)
    const double *B;          // solve: right-hand sides, n x m (ldb); X receives A^-1 B (n x m, ldx)
    int64_t ldb;
    int32_t k0;               // blocked elimination: steps before this panel (0 otherwise)
    int32_t inplace;          // init: W already holds the trailing block (no copy, header kept)
};

}  // namespace gj
