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
// Quarter table q[m][ny/2+1][nx/2+1] of a FULL table (plan dtype: dbl selects double2),
// with stats[0] = max |T[k] - T[|k1|, |k2|, k3]| and stats[1] = max |T[k]| (FP64 bit patterns)
hipError_t launch_quarter(const void* full, void* q, int nx, int ny, int m, int dbl, unsigned long long* stats,
                          hipStream_t s);
// y = (first ? 0 : y) + w x over n complex FP64 values (sums of kernel tables)
hipError_t launch_axpy64(const double2* x, double2* y, long long n, double w, int first, hipStream_t s);
// Radial-profile tables from the 2-D DFT of the hat basis (cached per geometry):
// hr[q][k2][k1], 0 <= k1 <= nx/2, 0 <= k2 <= ny/2, the real spectrum of basis[q] (tmp:
// nq ny (nx/2+1) double2 of scratch), then the FFC table folded into acc for profiles with
// M <= kProfileFoldMaxM and n_knots <= kProfileFoldMaxM (pht: 4 n_knots 16 double2).
constexpr int kProfileFoldMaxM = 64;
hipError_t launch_basis_dft(const double* basis, const double2* twx, const double2* twy, int nq, int nx, int ny,
                            double2* tmp, double* hr, hipStream_t s);
hipError_t launch_profile_fold(const double* prof, const double2* twm, const double* hr, int nq, int nx, int ny,
                               int m, int norm_mode, double2* pht, double2* acc, int first, hipStream_t s);
hipError_t launch_exp_gauss_samples(double sigma, int nx, int ny, int m, double* out, hipStream_t s);
hipError_t launch_profile_samples(const double* prof, int n_knots, double r_max, int nx, int ny, int m, double* out,
                                  hipStream_t s);

}  // namespace se2c
