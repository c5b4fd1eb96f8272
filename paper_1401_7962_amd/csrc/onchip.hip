// onchip.hip -- full-pivot Gauss-Jordan with the matrix held in registers.
//
// One matrix per 256-thread workgroup (kind 0, n <= 128) or per wavefront
// (kind 1, n <= 64).  The n x n array (the in-place [A|D] of eqs. 3-10) is
// distributed cyclically over a TR x TC thread grid: thread (tr, tc) holds
// rows a*TR + tr and columns b*TC + tc, EA x EB values in VGPRs.
//
// One step k (paper section 2):
//   1. the winner of the pivot search (Obs. 2-3) is already known from the
//      fused argmax of the previous step (largest |a| over the trailing block,
//      ties to the lowest row then column);
//   2. singular / non-finite test against the zero threshold (Obs. 2);
//   3. rows k,r and columns k,c are swapped physically: the owners of the four
//      lines stage them in LDS, together with the pivot row already divided by
//      the pivot (eq. 14, correctly rounded division, slot (k,k) = 1/p) and
//      the pivot column (the multipliers a_ik);
//   4. every element takes one fma with the staged row and column (eq. 15);
//      the pivot row is then overwritten with its scaled values;
//   5. while the new values are in registers, each thread scans its part of
//      the next trailing block in row-major order (so strict '>' keeps the
//      first maximum), and the workgroup reduces (|a|, row<<16|col).
// The determinant (eq. 13) is accumulated as an exact mantissa/exponent pair.
// The final depivoting (Obs. 3) is folded into the store: element (i, j) of
// the working array goes to X(g[i], h[j]), where g and h are the inverse
// permutations of the reversed swap sequence, built forward one swap per
// step.
#include "gj_device.h"

namespace gj {

template <typename T, int N, int NW>
struct CoreLds {
    T prow[N];     // new pivot row, divided by the pivot
    T pcol[N];     // new pivot column (multipliers)
    T newr[N];     // new row r  (= old row k, columns swapped)
    T newc[N];     // new column c (= old column k, rows swapped)
    int32_t g[N];  // destination row of working row i
    int32_t h[N];  // destination column of working column j
    Cand<T> red[NW];
    int32_t nfw[NW];
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

// Reduce (|a|, key) over the group.  Every thread ends with the same winner.
template <typename T, int N, int NW>
__device__ inline void group_argmax(Cand<T> &c, bool &nf, CoreLds<T, N, NW> &L, int t) {
    wave_argmax(c);
    int any_nf = __any(nf ? 1 : 0);
    if constexpr (NW == 1) {
        nf = any_nf != 0;
    } else {
        const int lane = t & (kWave - 1), w = t / kWave;
        if (lane == 0) {
            L.red[w] = c;
            L.nfw[w] = any_nf;
        }
        __syncthreads();
        Cand<T> best = L.red[0];
        int nfa = L.nfw[0];
#pragma unroll
        for (int x = 1; x < NW; ++x) {
            Cand<T> o = L.red[x];
            nfa |= L.nfw[x];
            if (better(o.a, o.key, best.a, best.key)) best = o;
        }
        c = best;
        nf = nfa != 0;
    }
}

// Scan this thread's part of the trailing block (rows and columns > k, < n)
// in row-major order; strict '>' keeps the first maximum.  The winning slot
// is tracked as the compile-time code a*EB+b so that no per-element key has
// to stay live across steps; the key is formed once at the end.
template <typename T, int TR, int TC, int EA, int EB>
__device__ __forceinline__ void scan_argmax(const T (&v)[EA][EB], int k, int n, int tr, int tc,
                                            Cand<T> &c, bool &nf) {
    using M = Num<T>;
    bool cok[EB];
#pragma unroll
    for (int b = 0; b < EB; ++b) {
        const int j = b * TC + tc;
        cok[b] = (j > k) && (j < n);
    }
    T best = (T)0;
    int code = -1;
    bool bad = false;
#pragma unroll
    for (int a = 0; a < EA; ++a) {
        const int i = a * TR + tr;
        const bool rok = (i > k) && (i < n);
#pragma unroll
        for (int b = 0; b < EB; ++b) {
            const T x = v[a][b];
            const bool ok = rok && cok[b];
            bad |= ok && !M::finite_(x);
            if (ok && M::abs_(x) > M::abs_(best)) {
                best = x;
                code = a * EB + b;
            }
        }
    }
    c.v = best;
    c.a = M::abs_(best);
    if (code >= 0) {
        const int i = (code / EB) * TR + tr, j = (code % EB) * TC + tc;
        c.key = ((uint32_t)i << 16) | (uint32_t)j;
    } else {
        c.key = 0xFFFFFFFFu;
    }
    nf = bad;
}

template <typename T, int TR, int TC, int EA, int EB, int NW>
__device__ __forceinline__ void gj_core(int t, const MatDesc md, const double *__restrict__ A,
                        double *__restrict__ X, int32_t *__restrict__ ipiv_all,
                        int32_t *__restrict__ jpiv_all, gj_result *__restrict__ res_all,
                        double zero_tol, double eps_default, int det_only,
                        CoreLds<T, TR * EA, NW> &L) {
    constexpr int N = TR * EA;
    static_assert(TR * EA == TC * EB, "square tiling");
    static_assert(TR * TC == NW * kWave, "thread grid");
    using M = Num<T>;
    const int n = md.n;
    const int tr = t / TC, tc = t % TC;
    int32_t *ipiv = ipiv_all + md.piv_off;
    int32_t *jpiv = jpiv_all + md.piv_off;
    gj_result *res = res_all + md.res_idx;

    T v[EA][EB];
#pragma unroll
    for (int a = 0; a < EA; ++a) {
        const int i = a * TR + tr;
#pragma unroll
        for (int b = 0; b < EB; ++b) {
            const int j = b * TC + tc;
            v[a][b] = (i < n && j < n) ? (T)A[md.a_off + (int64_t)i * md.lda + j] : (T)0;
        }
    }
    for (int x = t; x < N; x += TR * TC) {
        L.prow[x] = (T)0;
        L.pcol[x] = (T)0;
        L.g[x] = x;
        L.h[x] = x;
    }

    // pivot search of step 0 over the whole matrix
    Cand<T> c;
    bool nf = false;
    scan_argmax<T, TR, TC, EA, EB>(v, -1, n, tr, tc, c, nf);
    group_argmax(c, nf, L, t);

    const T tau = (zero_tol >= 0.0) ? (T)zero_tol : (T)n * (T)eps_default * c.a;
    DetAcc<T> det;
    det.init();
    int code = GJ_RES_OK, rank = n;

    for (int k = 0; k < n; ++k) {
        if (nf) { code = GJ_RES_NONFINITE; rank = k; break; }
        if (c.a == (T)0 || c.a < tau) { code = GJ_RES_SINGULAR; rank = k; break; }
        const int r = (int)(c.key >> 16), cc = (int)(c.key & 0xFFFFu);
        const T p = c.v;
        det.mul(p);
        if (r != k) det.sign = -det.sign;
        if (cc != k) det.sign = -det.sign;
        if (t == 0) {
            ipiv[k] = r;
            jpiv[k] = cc;
            int tmp = L.g[k]; L.g[k] = L.g[cc]; L.g[cc] = tmp;
            tmp = L.h[k]; L.h[k] = L.h[r]; L.h[r] = tmp;
        }
        const int ar = r / TR, trr = r % TR, ak = k / TR, trk = k % TR;
        const int bc = cc / TC, tcc = cc % TC, bk = k / TC, tck = k % TC;
        const T one = M::one();

        // stage the four swapped lines and the scaled pivot row (eq. 14)
        if (tr == trr) {
#pragma unroll
            for (int a = 0; a < EA; ++a) if (a == ar) {
#pragma unroll
                for (int b = 0; b < EB; ++b) {
                    const int jo = b * TC + tc;
                    if (jo < n) {
                        const int jn = (jo == cc) ? k : ((jo == k) ? cc : jo);
                        L.prow[jn] = ((jo == cc) ? one : v[a][b]) / p;
                    }
                }
            }
        }
        if (tr == trk) {
#pragma unroll
            for (int a = 0; a < EA; ++a) if (a == ak) {
#pragma unroll
                for (int b = 0; b < EB; ++b) {
                    const int jo = b * TC + tc;
                    if (jo < n) {
                        const int jn = (jo == cc) ? k : ((jo == k) ? cc : jo);
                        L.newr[jn] = v[a][b];
                    }
                }
            }
        }
        if (tc == tcc) {
#pragma unroll
            for (int b = 0; b < EB; ++b) if (b == bc) {
#pragma unroll
                for (int a = 0; a < EA; ++a) {
                    const int io = a * TR + tr;
                    if (io < n) {
                        const int in = (io == r) ? k : ((io == k) ? r : io);
                        L.pcol[in] = v[a][b];
                    }
                }
            }
        }
        if (tc == tck) {
#pragma unroll
            for (int b = 0; b < EB; ++b) if (b == bk) {
#pragma unroll
                for (int a = 0; a < EA; ++a) {
                    const int io = a * TR + tr;
                    if (io < n) {
                        const int in = (io == r) ? k : ((io == k) ? r : io);
                        L.newc[in] = v[a][b];
                    }
                }
            }
        }
        group_sync<NW>();

        // install the swapped row r and column c; clear column k (it becomes
        // fma(-q, 1/p, 0) below, the D column of eq. 15)
        if (tr == trr) {
#pragma unroll
            for (int a = 0; a < EA; ++a) if (a == ar) {
#pragma unroll
                for (int b = 0; b < EB; ++b) {
                    const int j = b * TC + tc;
                    if (j < n) v[a][b] = L.newr[j];
                }
            }
        }
        if (tc == tcc) {
#pragma unroll
            for (int b = 0; b < EB; ++b) if (b == bc) {
#pragma unroll
                for (int a = 0; a < EA; ++a) {
                    const int i = a * TR + tr;
                    if (i < n) v[a][b] = L.newc[i];
                }
            }
        }
        if (tc == tck) {
#pragma unroll
            for (int b = 0; b < EB; ++b) if (b == bk) {
#pragma unroll
                for (int a = 0; a < EA; ++a) v[a][b] = (T)0;
            }
        }

        // eq. 15 for every row, then the pivot row takes its scaled values
        T q[EA], pr[EB];
#pragma unroll
        for (int a = 0; a < EA; ++a) q[a] = L.pcol[a * TR + tr];
#pragma unroll
        for (int b = 0; b < EB; ++b) pr[b] = L.prow[b * TC + tc];
#pragma unroll
        for (int a = 0; a < EA; ++a)
#pragma unroll
            for (int b = 0; b < EB; ++b) v[a][b] = M::fma_(-q[a], pr[b], v[a][b]);
        if (tr == trk) {
#pragma unroll
            for (int a = 0; a < EA; ++a) if (a == ak) {
#pragma unroll
                for (int b = 0; b < EB; ++b) v[a][b] = pr[b];
            }
        }

        // fused pivot search for step k+1 over rows and columns > k
        if (k + 1 < n) {
            scan_argmax<T, TR, TC, EA, EB>(v, k, n, tr, tc, c, nf);
            group_argmax(c, nf, L, t);
        }
    }

    // ensure thread 0's last swaps of g/h are visible
    group_sync<NW>();
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
        for (int x = rank + t; x < n; x += TR * TC) {
            ipiv[x] = -1;
            jpiv[x] = -1;
        }
        if (t == 0) write_result_fail(res, code, rank);
    }
}

// LDS shared by the two task kinds (union by reinterpretation).
template <typename T>
struct OnchipShared {
    static constexpr size_t k0 = sizeof(CoreLds<T, 128, 4>);
    static constexpr size_t k1 = 4 * sizeof(CoreLds<T, 64, 1>);
    static constexpr size_t bytes = (k0 > k1 ? k0 : k1);
};

// Kind 0: one matrix, all four wavefronts.
template <typename T>
__device__ inline void run_kind0(unsigned char *smem, int t, const MatDesc &md, const double *A,
                                 double *X, int32_t *ipiv, int32_t *jpiv, gj_result *res,
                                 double zero_tol, double eps_default, int det_only) {
    if (md.n <= 32) {
        gj_core<T, 16, 16, 2, 2, 4>(t, md, A, X, ipiv, jpiv, res, zero_tol, eps_default, det_only,
                                    *reinterpret_cast<CoreLds<T, 32, 4> *>(smem));
    } else if (md.n <= 64) {
        gj_core<T, 16, 16, 4, 4, 4>(t, md, A, X, ipiv, jpiv, res, zero_tol, eps_default, det_only,
                                    *reinterpret_cast<CoreLds<T, 64, 4> *>(smem));
    } else {
        gj_core<T, 16, 16, 8, 8, 4>(t, md, A, X, ipiv, jpiv, res, zero_tol, eps_default, det_only,
                                    *reinterpret_cast<CoreLds<T, 128, 4> *>(smem));
    }
}

// Kind 1: one matrix per wavefront (n <= 64).
template <typename T>
__device__ inline void run_kind1(unsigned char *smem, int lane, int w, const MatDesc &md,
                                 const double *A, double *X, int32_t *ipiv, int32_t *jpiv,
                                 gj_result *res, double zero_tol, double eps_default, int det_only) {
    unsigned char *Lw = smem + (size_t)w * sizeof(CoreLds<T, 64, 1>);
    if (md.n <= 8) {
        gj_core<T, 8, 8, 1, 1, 1>(lane, md, A, X, ipiv, jpiv, res, zero_tol, eps_default, det_only,
                                  *reinterpret_cast<CoreLds<T, 8, 1> *>(Lw));
    } else if (md.n <= 16) {
        gj_core<T, 8, 8, 2, 2, 1>(lane, md, A, X, ipiv, jpiv, res, zero_tol, eps_default, det_only,
                                  *reinterpret_cast<CoreLds<T, 16, 1> *>(Lw));
    } else if (md.n <= 32) {
        gj_core<T, 8, 8, 4, 4, 1>(lane, md, A, X, ipiv, jpiv, res, zero_tol, eps_default, det_only,
                                  *reinterpret_cast<CoreLds<T, 32, 1> *>(Lw));
    } else {
        gj_core<T, 8, 8, 8, 8, 1>(lane, md, A, X, ipiv, jpiv, res, zero_tol, eps_default, det_only,
                                  *reinterpret_cast<CoreLds<T, 64, 1> *>(Lw));
    }
}

// Persistent kernel: workgroups take tasks from an atomic queue until it is
// empty; tasks are ordered by decreasing cost on the host.  With mats ==
// nullptr the kernel inverts the single matrix passed by value (workgroup 0).
template <typename T>
__global__ void __launch_bounds__(256)
gj_onchip_kernel(const MatDesc *__restrict__ mats, const OnchipTask *__restrict__ tasks,
                 int ntasks, uint32_t *__restrict__ queue, const MatDesc single,
                 const double *__restrict__ A, double *__restrict__ X, int32_t *__restrict__ ipiv,
                 int32_t *__restrict__ jpiv, gj_result *__restrict__ res, double zero_tol,
                 double eps_default, int det_only, const int32_t *__restrict__ run_flag) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[OnchipShared<T>::bytes];
    __shared__ int s_task;
    const int t = threadIdx.x;
    if (run_flag && *run_flag == 0) return;
    if (mats == nullptr) {
        if (blockIdx.x == 0)
            run_kind0<T>(smem, t, single, A, X, ipiv, jpiv, res, zero_tol, eps_default, det_only);
        return;
    }
    for (;;) {
        if (t == 0) s_task = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int id = s_task;
        __syncthreads();
        if (id >= ntasks) break;
        const OnchipTask task = tasks[id];
        if (task.kind == 0) {
            const MatDesc md = mats[task.m[0]];
            run_kind0<T>(smem, t, md, A, X, ipiv, jpiv, res, zero_tol, eps_default, det_only);
        } else {
            const int w = t / kWave, lane = t % kWave;
            const int mi = task.m[w];
            if (mi >= 0) {
                const MatDesc md = mats[mi];
                run_kind1<T>(smem, lane, w, md, A, X, ipiv, jpiv, res, zero_tol, eps_default,
                             det_only);
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

hipError_t launch_onchip(bool fp32, const MatDesc *mats, const OnchipTask *tasks, int ntasks,
                         uint32_t *queue, const MatDesc &single, int grid, const double *A,
                         double *X, int32_t *ipiv, int32_t *jpiv, gj_result *res, double zero_tol,
                         double eps_default, int det_only, const int32_t *run_flag,
                         hipStream_t s) {
    if (mats) {
        hipError_t e = launch_zero_u32(queue, 1, s);
        if (e != hipSuccess) return e;
    }
    if (fp32)
        hipLaunchKernelGGL(gj_onchip_kernel<float>, dim3(grid), dim3(256), 0, s, mats, tasks,
                           ntasks, queue, single, A, X, ipiv, jpiv, res, zero_tol, eps_default,
                           det_only, run_flag);
    else
        hipLaunchKernelGGL(gj_onchip_kernel<double>, dim3(grid), dim3(256), 0, s, mats, tasks,
                           ntasks, queue, single, A, X, ipiv, jpiv, res, zero_tol, eps_default,
                           det_only, run_flag);
    return hipGetLastError();
}

}  // namespace gj
