// gj_launch.h -- host-side launchers of the libgj kernels (internal).
#pragma once

#include "gj_device.h"

namespace gj {

hipError_t launch_zero_u32(uint32_t *p, int count, hipStream_t s);

// on-chip task classes for batches: 0 = (kind 0, E 8, n in 65..128),
// 1..4 = (kind 1, E 8/4/2/1, n in 33..64 / 17..32 / 9..16 / 1..8)
constexpr int kOnchipClasses = 5;
int onchip_class_of(int n, bool single);
int onchip_class_kind(int c);
hipError_t launch_onchip_class(bool fp32, int cls, const MatDesc *mats, const OnchipTask *tasks,
                               int ntasks, uint32_t *queue, const MatDesc &single, const double *A,
                               double *X, int32_t *ipiv, int32_t *jpiv, gj_result *res,
                               double zero_tol, double eps_default, int det_only,
                               const int32_t *run_flag, hipStream_t s);

hipError_t launch_onchip(bool fp32, const MatDesc *mats, const OnchipTask *tasks, int ntasks,
                         uint32_t *queue, const MatDesc &single, int grid, const double *A,
                         double *X, int32_t *ipiv, int32_t *jpiv, gj_result *res, double zero_tol,
                         double eps_default, int det_only, const int32_t *run_flag,
                         hipStream_t s);

hipError_t launch_big(bool fp32, int nt, const BigDesc *descs, const int2 *bmap,
                      const BigDesc &single, const int *grid_per_step, int grid_init,
                      int grid_finish, int max_n, int gather_grid, double zero_tol,
                      double eps_default, int det_only, void *const *events,
                      const int32_t *run_flag, hipStream_t s);

struct GemmArgs {
    int M, N, K;
    const double *A;
    int64_t lda;
    const double *B;
    int64_t ldb;
    const double *C;
    int64_t ldc;
    double *D;
    int64_t ldd;
    double alpha, beta, gamma;
    double *norm_partials;
    const int32_t *run_flag;
};
int gemm_tiles(int M, int N);
hipError_t launch_gemm_f64(const GemmArgs &g, hipStream_t s);

// refinement path (refine.hip)
size_t refine_ctl_bytes();
const int32_t *ctl_run_ns(const void *c);
const int32_t *ctl_run_fallback(const void *c);
const int32_t *ctl_run_det(const void *c);
const int32_t *ctl_copy_back(const void *c);
const int32_t *ctl_always(const void *c);
hipError_t launch_refine_start(const gj_result *res32, void *ctl, hipStream_t s);
hipError_t launch_refine_resid0(const double *partials, int np, void *ctl, hipStream_t s);
hipError_t launch_refine_after_update(const double *partials, int np, void *ctl, int it,
                                      int max_iters, double stall, hipStream_t s);
hipError_t launch_refine_finish(void *ctl, double accept, int det_wanted, hipStream_t s);
hipError_t launch_copy_flagged(const double *src, int64_t lds, double *dst, int64_t ldd, int n,
                               const int32_t *flag, hipStream_t s);
hipError_t launch_fallback_mark(gj_result *res, const void *ctl, hipStream_t s);
hipError_t launch_perms_from_pivots(const int32_t *ipiv, const int32_t *jpiv, int n, int32_t *rows,
                                    int32_t *cols, const int32_t *flag, hipStream_t s);
hipError_t launch_gather_perm(const double *A, int64_t lda, const int32_t *rows, const int32_t *cols,
                              int n, double *B, int64_t ldb, const int32_t *flag, hipStream_t s);
hipError_t launch_det_combine(const gj_result *blocks, int nblocks, const int32_t *ipiv,
                              const int32_t *jpiv, int n, gj_result *res, void *ctl, hipStream_t s);
hipError_t launch_refine_iters(gj_result *res, const void *ctl, hipStream_t s);
int sumsq_blocks(int n);
hipError_t launch_sumsq(const double *M, int64_t ld, int n, double *partials, hipStream_t s);
hipError_t launch_resid(const double *pr, int nr, const double *pa, int na, const double *px, int nx,
                        gj_result *res, hipStream_t s);

}  // namespace gj
