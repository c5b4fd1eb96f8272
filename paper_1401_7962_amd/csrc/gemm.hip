// gemm.hip -- GEMM on the matrix cores: FP64 (v_mfma_f64_16x16x4f64) and
// FP32 (v_mfma_f32_16x16x4f32, for the delayed updates of the FP32
// elimination).
//
//   D = alpha * (A B) + beta * C + gamma * I        (row-major, FP64)
//
// Used where the method really is a dense contraction: the Newton-Schulz
// refinement (R = I - A X and X + X R) and the Schur-complement updates of
// the FP64 determinant.  Optionally writes, per workgroup, the sum of squares
// of the D tile it stored (for ||R||_F without a second pass), and skips all
// work when a device-side run flag is 0 (so that a fixed launch sequence can
// be captured in a HIP graph while the iteration count stays data-dependent).
//
// Tiling: 256 threads = 4 wavefronts in a 2 x 2 grid; workgroup tile
// 128 x 128, wavefront tile 64 x 64 = 4 x 4 MFMA blocks of 16 x 16, K staged
// through LDS 16 at a time with a register prefetch of the next K slice.
// Workgroups are numbered so that the ones resident on the same XCD (the
// hardware deals workgroups round-robin over 8 XCDs) take neighbouring tiles
// of the same row panel of A, which their shared L2 then serves.
#include "gj_launch.h"

// GemmArgs (gj_launch.h): C may alias D and is unused when beta == 0;
// norm_partials receives one sum of squares of the stored D per workgroup
// (null: none); run_flag null or pointing at a non-zero value lets it run.

namespace gj {


namespace {

constexpr int BM = 128, BN = 128, BK = 16, NTH = 256;
constexpr int LDA_S = BM + 2;  // LDS row pitch (doubles), padded against bank conflicts
constexpr int LDB_S = BN + 2;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// One 16 x 16 x 4 MFMA step and the accumulator layout of each precision:
// register r of lane l holds column l % 16 and row row(l / 16, r) of the
// 16 x 16 block (FP64: l/16 + 4r; FP32: 4 (l/16) + r).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
    using acc_t = d4;
    __device__ static acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lk, int r) { return lk + 4 * r; }
};
template <> struct Mfma<float> {
    using acc_t = f4;
    __device__ static acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lk, int r) { return 4 * lk + r; }
};

// One 128 x 128 tile of D.  `b` is the tile index within the problem,
// `part` the slot of its norm partial.
//
// The K loop is double-buffered in LDS: while the wavefronts multiply slice
// kt out of one buffer, the next slice (already in registers) is written to
// the other, and a single barrier per slice separates the two roles.  Global
// reads go through the global address space (not FLAT), so that waiting for
// an LDS read never waits for the prefetch of the next slice as well.
template <typename T>
__device__ __forceinline__ void gemm_tile(const GemmArgsT<T> &g, int b, int part) {
    using MF = Mfma<T>;
    __shared__ T As[2][BK][LDA_S];  // As[buf][k][m]
    __shared__ T Bs[2][BK][LDB_S];  // Bs[buf][k][n]
    __shared__ double s_red[NTH / kWave];

    const int tiles_n = (g.N + BN - 1) / BN;
    const int tm = b / tiles_n, tn = b % tiles_n;
    const int m0 = tm * BM, n0 = tn * BN;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
    const gptr<const T> gA = glb(g.A), gB = glb(g.B);

    typename MF::acc_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] = (T)0;

    // global -> register staging: A tile 128 x 16 (thread: row t/2, 8 k's),
    // B tile 16 x 128 (thread: k t/16, 8 columns)
    const int a_row = t >> 1, a_k0 = (t & 1) * 8;
    const int b_k = t >> 4, b_c0 = (t & 15) * 8;
    T ra[8], rb[8];
    auto load_tile = [&](int k0) {
        const int gm = m0 + a_row;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int gk = k0 + a_k0 + e;
            ra[e] = (gm < g.M && gk < g.K) ? gA[(int64_t)gm * g.lda + gk] : (T)0;
        }
        const int gk = k0 + b_k;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int gn = n0 + b_c0 + e;
            rb[e] = (gk < g.K && gn < g.N) ? gB[(int64_t)gk * g.ldb + gn] : (T)0;
        }
    };
    auto store_tile = [&](int buf) {
#pragma unroll
        for (int e = 0; e < 8; ++e) As[buf][a_k0 + e][a_row] = ra[e];
#pragma unroll
        for (int e = 0; e < 8; ++e) Bs[buf][b_k][b_c0 + e] = rb[e];
    };

    const int nk = (g.K + BK - 1) / BK;
    load_tile(0);
    store_tile(0);
    __syncthreads();
    const int li = lane & 15, lk = lane >> 4;
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) load_tile((kt + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            T fa[4], fb[4];
#pragma unroll
            for (int f = 0; f < 4; ++f) fa[f] = As[cur][kk + lk][wm * 64 + f * 16 + li];
#pragma unroll
            for (int f = 0; f < 4; ++f) fb[f] = Bs[cur][kk + lk][wn * 64 + f * 16 + li];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = MF::step(fa[i], fb[j], acc[i][j]);
        }
        if (kt + 1 < nk) store_tile(cur ^ 1);
        __syncthreads();
    }

    // epilogue: accumulator register r of lane l holds column l % 16 and row
    // MF::row(l / 16, r) of its 16 x 16 block
    double ssq = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = n0 + wn * 64 + j * 16 + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 64 + i * 16 + MF::row(lk, r);
                if (row < g.M && col < g.N) {
                    T v = (T)g.alpha * acc[i][j][r];
                    if (g.beta != 0.0) v = fma((T)g.beta, glb(g.C)[(int64_t)row * g.ldc + col], v);
                    if (row == col) v += (T)g.gamma;
                    glb(g.D)[(int64_t)row * g.ldd + col] = v;
                    ssq = fma((double)v, (double)v, ssq);
                }
            }
        }
    }
    if (g.norm_partials) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) ssq += __shfl_xor(ssq, off, kWave);
        if (lane == 0) s_red[w] = ssq;
        __syncthreads();
        if (t == 0) glb(g.norm_partials)[part] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
    }
}

__global__ void __launch_bounds__(NTH, 2)
gemm_f64_kernel(const GemmArgs g) {
    if (g.run_flag && *g.run_flag == 0) return;
    const int ntiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
    // XCD-aware renumbering: hardware workgroup b runs on XCD b % 8
    int b = blockIdx.x;
    if (ntiles % 8 == 0) b = (b % 8) * (ntiles / 8) + b / 8;
    gemm_tile<double>(g, b, blockIdx.x);
}

__global__ void __launch_bounds__(NTH, 2)
gemm_f32_kernel(const GemmArgsT<float> g) {
    if (g.run_flag && *g.run_flag == 0) return;
    const int ntiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
    int b = blockIdx.x;
    if (ntiles % 8 == 0) b = (b % 8) * (ntiles / 8) + b / 8;
    gemm_tile<float>(g, b, blockIdx.x);
}

// Many independent products in one launch: workgroup -> (problem, tile).
__global__ void __launch_bounds__(NTH, 2)
gemm_f64_grouped_kernel(const GemmArgs *__restrict__ probs, const int2 *__restrict__ tilemap) {
    const int2 pt = tilemap[blockIdx.x];
    const GemmArgs g = probs[pt.x];
    if (g.run_flag && *g.run_flag == 0) return;
    gemm_tile<double>(g, pt.y, pt.y);
}

}  // namespace

int gemm_tiles(int M, int N) { return ((M + BM - 1) / BM) * ((N + BN - 1) / BN); }

hipError_t launch_gemm_f64_grouped(const GemmArgs *probs, const int2 *tilemap, int ntiles,
                                   hipStream_t s) {
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(gemm_f64_grouped_kernel, dim3(ntiles), dim3(NTH), 0, s, probs, tilemap);
    return hipGetLastError();
}

hipError_t launch_gemm_f64(const GemmArgs &g, hipStream_t s) {
    const int tiles = gemm_tiles(g.M, g.N);
    if (tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(gemm_f64_kernel, dim3(tiles), dim3(NTH), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_gemm_f32(const GemmArgsT<float> &g, hipStream_t s) {
    const int tiles = gemm_tiles(g.M, g.N);
    if (tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(gemm_f32_kernel, dim3(tiles), dim3(NTH), 0, s, g);
    return hipGetLastError();
}

}  // namespace gj
