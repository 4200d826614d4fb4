// Gradient kernels (see grad.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace se2c {

hipError_t launch_unpack_tables(const void* zre, const void* zim, void* ta, void* tb, int nx, int ny, int m, bool dbl,
                                hipStream_t s);
hipError_t launch_accumulate_pair(const void* zre, const void* zim, const void* ta, const void* tb, void* accre,
                                  void* accim, int nx, int ny, int m, double scale, int first, bool dbl,
                                  hipStream_t s);
// points per split of the profile-gradient contraction
constexpr int kProfileChunk = 64;
int profile_grad_splits(long long npts);
// basis[q][j][i]: hat function q (knots r_q = q r_max / (n_knots - 1)) at |x_ij|, lattice-periodized
hipError_t launch_profile_basis(double* basis, int n_knots, double r_max, int nx, int ny, hipStream_t s);
// grad[q][l] = sum_b sum_p basis[q][p] g_b[l][p]; G: npts*m doubles, part: splits*n_knots*m doubles
hipError_t launch_profile_grad(const void* g, int batch, bool dbl, int n_knots, int nx, int ny, int m,
                               const double* basis, double* G, double* part, double* grad, hipStream_t s);

}  // namespace se2c
