// gj_launch.h -- host-side launchers of the libgj kernels (internal).
#pragma once

#include "gj_device.h"

namespace gj {

hipError_t launch_zero_u32(uint32_t *p, int count, hipStream_t s);

hipError_t launch_onchip(bool fp32, const MatDesc *mats, const OnchipTask *tasks, int ntasks,
                         uint32_t *queue, const MatDesc &single, int grid, const double *A,
                         double *X, int32_t *ipiv, int32_t *jpiv, gj_result *res, double zero_tol,
                         double eps_default, int det_only, hipStream_t s);

hipError_t launch_big(bool fp32, int nt, const BigDesc *descs, const int2 *bmap,
                      const BigDesc &single, const int *grid_per_step, int grid_init,
                      int grid_finish, int max_n, int gather_grid, double zero_tol,
                      double eps_default, int det_only, void *const *events, hipStream_t s);

}  // namespace gj
