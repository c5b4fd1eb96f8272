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

// Argmax candidate: largest |a|, ties to the smallest key.  key packs
// (row << 16 | col) of the current matrix, so unsigned order is row-major
// order.
template <typename T> struct Cand {
    T a;         // |value|, -1 when the thread has no candidate
    T v;         // signed value
    uint32_t key;
};

template <typename T>
__device__ inline bool better(T a1, uint32_t k1, T a2, uint32_t k2) {
    return (a1 > a2) || (a1 == a2 && k1 < k2);
}

template <typename T>
__device__ inline void wave_argmax(Cand<T> &c) {
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) {
        T oa = __shfl_xor(c.a, off, kWave);
        T ov = __shfl_xor(c.v, off, kWave);
        uint32_t ok = (uint32_t)__shfl_xor((int)c.key, off, kWave);
        if (better(oa, ok, c.a, c.key)) {
            c.a = oa;
            c.v = ov;
            c.key = ok;
        }
    }
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
};

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
    int32_t n, R, nblk, tpr;  // order, rows per workgroup, workgroups, threads per row
};

}  // namespace gj
