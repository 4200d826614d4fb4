// Sampling of synthetic fields on Omega_L (the grid of paper Sec. 3.2, eq. (OmL)).
//
// f(x, theta) = sum_b w_b G(x - c_bx) G(y - c_by) exp(kappa cos(theta - theta0_b)),
// G(u) = sum_{l=-3..3} exp(-(u + l)^2 / (2 s^2))  (lattice periodization, eq. (TH),
// truncated to the images that matter for s <= 0.1).  Evaluated in FP64 and rounded.
#include <hip/hip_runtime.h>

#include "sample.hpp"

namespace se2c {

// 1-D profiles per bump: prof[b] = gx[nx] | gy[ny] | h[m] (h includes the weight).
__global__ void bump_profiles_kernel(const double* params, int nb, double s, double kappa, int nx, int ny, int m,
                                     double* prof) {
    const int len = nx + ny + m;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < (long long)nb * len;
         idx += (long long)gridDim.x * blockDim.x) {
        const int b = (int)(idx / len);
        const int i = (int)(idx - (long long)b * len);
        const double cx = params[4 * b], cy = params[4 * b + 1], t0 = params[4 * b + 2], w = params[4 * b + 3];
        double v = 0.0;
        if (i < nx + ny) {
            const int L = i < nx ? nx : ny;
            const int k = i < nx ? i : i - nx;
            const double u = -0.5 + (double)k / L - (i < nx ? cx : cy);
            for (int l = -3; l <= 3; ++l) {
                const double d = u + l;
                v += exp(-(d * d) / (2.0 * s * s));
            }
        } else {
            const int l = i - nx - ny;
            v = w * exp(kappa * cos(2.0 * M_PI * (double)l / m - t0));
        }
        prof[idx] = v;
    }
}

template <typename T>
__global__ void bump_sum_kernel(const double* prof, int nb, int nx, int ny, int m, T* out) {
    const int len = nx + ny + m;
    const long long n = (long long)nx * ny * m;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(idx % nx);
        const int j = (int)((idx / nx) % ny);
        const int l = (int)(idx / ((long long)nx * ny));
        double acc = 0.0;
        for (int b = 0; b < nb; ++b) {
            const double* pb = prof + (long long)b * len;
            acc += pb[nx + ny + l] * pb[nx + j] * pb[i];
        }
        out[idx] = (T)acc;
    }
}

hipError_t launch_sample_bumps(const double* params, int nb, double s, double kappa, int nx, int ny, int m,
                               double* prof, void* out, bool dbl, hipStream_t st) {
    hipLaunchKernelGGL(bump_profiles_kernel, dim3(256), dim3(256), 0, st, params, nb, s, kappa, nx, ny, m, prof);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (dbl)
        hipLaunchKernelGGL(bump_sum_kernel<double>, dim3(4096), dim3(256), 0, st, prof, nb, nx, ny, m,
                           reinterpret_cast<double*>(out));
    else
        hipLaunchKernelGGL(bump_sum_kernel<float>, dim3(4096), dim3(256), 0, st, prof, nb, nx, ny, m,
                           reinterpret_cast<float*>(out));
    return hipGetLastError();
}

}  // namespace se2c
