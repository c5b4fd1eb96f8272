// gj_launch.h -- host-side launchers of the libgj kernels (internal).
#pragma once

#include "gj_device.h"

namespace gj {

hipError_t launch_zero_u32(uint32_t *p, int count, hipStream_t s);

// integer environment override (dflt when unset or unparsable)
int env_int(const char *name, int dflt);

// on-chip task classes: c = 0..7 is kind 0 (one matrix per workgroup) with
// E = 8 - c register blocks per thread and dimension (n <= 16 E); c = 8..15
// is kind 1 (one matrix per wavefront) with E = 16 - c (n <= 8 E).
// onchip_class_of returns a class index in [0, kOnchipClasses), or -1.
constexpr int kOnchipClasses = 16;
int onchip_class_of(int n, bool single);
int onchip_class_kind(int c);
// det_only bit 1 (kOnchipStaticPivots, FP64 only): step k pivots on element
// (k, k), no search (rows and columns already in pivot order).
constexpr int kOnchipStaticPivots = 2;
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

// Streaming path: init, one step launch per k, finish, gather.  nt_loads:
// nontemporal row loads; full: the chunk count 1-8 that every matrix's rows
// fill exactly, else 0 (below 8: rule 0, nt < 1024, not counted, no rhs);
// counted: some descriptor leaves work units to the
// per-step counter (needs 8 full chunks and nt < 1024); rhs: a solve whose
// B is an extra partial register chunk after A's 8 full ones (FP64,
// nt < 1024, not counted); rule: pivot rule of every descriptor (0 full;
// 1, 2 need FP64 and none of full, counted, rhs).
hipError_t launch_big(bool fp32, int nt, bool nt_loads, int full, bool counted, bool rhs, int rule,
                      const BigDesc *descs,
                      const int2 *bmap,
                      const BigDesc &single, const int *grid_per_step, int grid_init,
                      int grid_finish, int max_n, int gather_grid, double zero_tol,
                      double eps_default, int det_only, void *const *events,
                      const int32_t *run_flag, hipStream_t s);

// blocked elimination (blocked.hip)
hipError_t launch_blk_init_perm(int32_t *prow, int32_t *pcol, int n, hipStream_t s);
hipError_t launch_blk_panel_end(bool fp32, const BigHdr *hdr, const int32_t *rl, const int32_t *cl,
                                int m, int32_t *rphys, int32_t *cphys, StepRec *steps_k0, int nbp,
                                int k0, const void *W, void *W2, int64_t ldw, int n, void *tA,
                                int ldta, void *tB, int64_t ldtb, const int32_t *prow_old,
                                const int32_t *pcol_old, int32_t *prow_new, int32_t *pcol_new,
                                hipStream_t s);
// X null: the record, pivots and position maps only
hipError_t launch_blk_finish(bool fp32, const BigHdr *hdr, const StepRec *steps, int n,
                             int32_t *ipiv, int32_t *jpiv, gj_result *res, const int32_t *prow,
                             const int32_t *pcol, int32_t *rowinv, int32_t *colinv, const void *W,
                             int64_t ldw, double *X, int64_t ldx, hipStream_t s);

template <typename T>
struct GemmArgsT {
    int M, N, K;
    const T *A;
    int64_t lda;
    const T *B;
    int64_t ldb;
    const T *C;
    int64_t ldc;
    T *D;
    int64_t ldd;
    double alpha, beta, gamma;
    double *norm_partials;
    const int32_t *run_flag;
};
using GemmArgs = GemmArgsT<double>;
int gemm_tiles(int M, int N);
hipError_t launch_gemm_f64(const GemmArgs &g, hipStream_t s);
// the same product in FP32 (v_mfma_f32_16x16x4f32; FP32 accumulation)
hipError_t launch_gemm_f32(const GemmArgsT<float> &g, hipStream_t s);
// grouped: workgroup b computes tile tilemap[b].y of problem probs[tilemap[b].x]
// (norm partial slot = tile index within the problem)
hipError_t launch_gemm_f64_grouped(const GemmArgs *probs, const int2 *tilemap, int ntiles,
                                   hipStream_t s);

// refinement path (refine.hip)
// Per-matrix refinement state (device).  A single call has one; a batch has
// one per member, all driven by the same launches.
struct RefineCtl {
    int32_t run_ns;        // refinement still running
    int32_t run_fallback;  // plain FP64 elimination needed
    int32_t run_det;       // FP64 block determinant needed
    int32_t updates;       // Newton-Schulz updates kept
    int32_t final_buf;     // 0: iterate in X, 1: iterate in the workspace copy
    int32_t copy_back;     // 1: copy the workspace iterate into X
    int32_t always;        // constant 1 (a run flag that is always set)
    int32_t nparts;        // GEMM norm partials of this matrix
    double r;              // ||R||_F of the kept iterate
    double r0;             // ||R_0||_F
    double *partials;
    gj_result *res;
    int32_t run_acc;       // accurate-residual phase still running
    int32_t acc_updates;   // updates kept in that phase
    double r_acc;          // ||R||_F of the last accurate residual
    unsigned long long xmax_bits;   // max |X| of the current iterate, as bits (non-negative)
};

// Per-matrix buffers of the refined path (device pointers).
struct RefMember {
    const double *A;
    int64_t lda;
    double *X;
    int64_t ldx;
    double *Xw;                  // second iterate (ld n)
    double *B;                   // permuted copy for the determinant (ld n)
    int32_t *ipiv, *jpiv;
    const int32_t *rows, *cols;  // FP32 pivot order as permutations
    int32_t *rows_buf, *cols_buf;  // non-null: fill rows/cols by replaying the swaps
    gj_result *blockres;         // one record per diagonal block
    int32_t n, nblocks;
};
size_t refine_ctl_bytes();
size_t refine_member_bytes();
const int32_t *ctl_run_ns(const void *c);
const int32_t *ctl_run_fallback(const void *c);
const int32_t *ctl_run_det(const void *c);
const int32_t *ctl_copy_back(const void *c);
const int32_t *ctl_always(const void *c);
void *ctl_at(void *c, int m);
hipError_t launch_refine_bind(void *ctl, gj_result *res, double *partials, int nparts, hipStream_t s);
hipError_t launch_refine_start(void *ctls, int count, hipStream_t s);
hipError_t launch_refine_resid0(void *ctls, int count, hipStream_t s);
hipError_t launch_refine_after_update(void *ctls, int count, int it, int max_iters, double stall,
                                      hipStream_t s);
hipError_t launch_refine_finish(void *ctls, int count, double accept, int det_wanted, hipStream_t s);
hipError_t launch_copy_back(const RefMember *mem, const RefMember &single, void *ctls, int count,
                            int row_blocks, hipStream_t s);
hipError_t launch_fallback_mark(void *ctls, int count, hipStream_t s);
hipError_t launch_perms_from_pivots(const RefMember *mem, const RefMember &single, void *ctls,
                                    int count, hipStream_t s);
hipError_t launch_gather_perm(const RefMember *mem, const RefMember &single, void *ctls, int count,
                              int row_blocks, hipStream_t s);
hipError_t launch_det_combine(const RefMember *mem, const RefMember &single, void *ctls, int count,
                              hipStream_t s);
hipError_t launch_refine_iters(void *ctls, int count, hipStream_t s);
// accurate-residual phase (single matrix): see accurate.hip
const int32_t *ctl_run_acc(const void *c);
hipError_t launch_acc_prepare(void *ctl, int enabled, hipStream_t s);
hipError_t launch_slice_rows(const double *A, int64_t lda, int n, double *S, int beta,
                             const int32_t *run, hipStream_t s);
hipError_t launch_slice_global(const double *X, int64_t ldx, int n, void *ctl, double *S, int beta,
                               hipStream_t s);
hipError_t launch_acc_check(void *ctl, int j, hipStream_t s);
hipError_t launch_acc_copy(const double *src, int n, double *X, int64_t ldx, const void *ctl,
                           hipStream_t s);
hipError_t launch_acc_finish(void *ctl, hipStream_t s);
int sumsq_blocks(int n);
hipError_t launch_sumsq(const double *M, int64_t ld, int n, double *partials, hipStream_t s);
hipError_t launch_resid(const double *pr, int nr, const double *pa, int na, const double *px, int nx,
                        gj_result *res, hipStream_t s);

}  // namespace gj
