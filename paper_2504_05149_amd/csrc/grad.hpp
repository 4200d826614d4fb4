// Gradient kernels (see grad.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace se2c {

hipError_t launch_unpack_tables(const void* zre, const void* zim, void* ta, void* tb, int nx, int ny, int m, bool dbl,
                                hipStream_t s);
hipError_t launch_accumulate_pair(const void* zre, const void* zim, const void* ta, const void* tb, void* accre,
                                  void* accim, int nx, int ny, int m, double scale, int first, bool dbl,
                                  hipStream_t s);
hipError_t launch_profile_grad(const void* g, int batch, bool dbl, int n_knots, double r_max, int nx, int ny, int m,
                               double* basis, double* G, double* grad, hipStream_t s);

}  // namespace se2c
