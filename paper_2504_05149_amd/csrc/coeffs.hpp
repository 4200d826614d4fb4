// FP64 coefficient-table generation (device launchers).
#pragma once
#include <hip/hip_runtime.h>

#define SE2C_GAUSS_IMAGES 3    // lattice images per axis for periodized Gaussians
#define SE2C_PROFILE_IMAGES 2  // lattice images per axis for radial profiles: support r_max + h <= 2 < 2.5

namespace se2c {

struct SepKernelParams {
    double sigma, kappa, theta0;
    double ive0;  // I0(kappa) * exp(-kappa), for the continuous normalisation
    int norm;     // 0 discrete mass, 1 continuous Haar mass, 2 none (raw samples)
};

hipError_t launch_sep_factor(const SepKernelParams& kp, int nx, int ny, int m, double2* acc64, int first,
                             hipStream_t s);
hipError_t launch_full_fold(const double* re, const double* im, double2* acc, long long n, int nx, int ny,
                            int norm_mode, int first, hipStream_t s);
hipError_t launch_full_fold_sep(const double2* sep, double2* acc, long long n, int nx, int ny, int first,
                                hipStream_t s);
hipError_t launch_round(const double2* src, void* dst, long long n, int dbl, hipStream_t s);
hipError_t launch_exp_gauss_samples(double sigma, int nx, int ny, int m, double* out, hipStream_t s);
hipError_t launch_profile_samples(const double* prof, int n_knots, double r_max, int nx, int ny, int m, double* out,
                                  hipStream_t s);

}  // namespace se2c
