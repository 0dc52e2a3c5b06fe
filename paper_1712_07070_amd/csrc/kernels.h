// Internal launch wrappers of libhydro (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hydro_device.h"

namespace gh {

template <typename T>
hipError_t launch_mhm_fwd(const T* U_pad, T* U_out, int64_t n_groups, int ghost, const Gas<T>& gas,
                          const double* dt_dev, double dx, int first_order, int ws, int* n_bad,
                          hipStream_t stream);

template <typename T>
hipError_t launch_fill_ghosts(const T* level, T* U_pad, int ngx, int ngy, int ngz, int ghost, const int bc[6],
                              hipStream_t stream);

template <typename T>
hipError_t launch_cfl_dt(const T* U_pad, int64_t n_groups, int ghost, double dx, double gamma, double c_cfl,
                         double* dt_patch, double* dt_min, hipStream_t stream);

}  // namespace gh
