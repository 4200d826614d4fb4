// Field sampling on the grid (see sample.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace se2c {
hipError_t launch_sample_bumps(const double* params, int nb, double s, double kappa, int nx, int ny, int m,
                               double* prof, void* out, bool dbl, hipStream_t st);
}
