// Kernels for gradients of the convolutional finite Fourier series.
//
// field tables  T_f[k] = (-1)^{k1+k2} F^[k] / n (eq. (FkLv)) of real fields, two at a
//               time: the complex FFT of z = f_a + i f_b gives Z^ = F_a^ + i F_b^, and
//               F_a^[k] = (Z^[k] + conj Z^[-k]) / 2, F_b^[k] = (Z^[k] - conj Z^[-k]) / 2i.
//               With these tables the kernel gradient is an adjoint apply:
//               dL/dP = Re S_K[g, conj(f^)] (d/dP of out = sum_k f^ rho^ phi_k with
//               rho^ = (-1)^{k1+k2} P^ / n).
// profile grad  dL/dprof[q][l] = sum_b sum_{j,i} H_q[j,i] dL/dP_b[l][j][i], H_q the
//               lattice-periodized hat basis in r = |x| (transpose of the radial-profile
//               sample expansion); FP64, deterministic (tree reductions, no atomics).
#include <hip/hip_runtime.h>

#include "coeffs.hpp"
#include "grad.hpp"

namespace se2c {

template <typename T>
__global__ void unpack_tables_kernel(const T* zre, const T* zim, void* ta, void* tb, int nx, int ny, int m) {
    using C2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
    const long long n = (long long)nx * ny * m;
    const T inv = (T)(1.0 / (double)n);
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int kx = (int)(idx % nx);
        const int ky = (int)((idx / nx) % ny);
        const int kt = (int)(idx / ((long long)nx * ny));
        const int mx = (nx - kx) % nx, my = (ny - ky) % ny, mt = (m - kt) % m;
        const long long midx = ((long long)mt * ny + my) * nx + mx;
        const T zr = zre[idx], zi = zim[idx];
        const T cr = zre[midx], ci = -zim[midx];  // conj Z^[-k]
        const T s = ((kx + ky) & 1) ? -inv : inv;
        C2 a, b;
        a.x = (T)0.5 * (zr + cr) * s;
        a.y = (T)0.5 * (zi + ci) * s;
        // (z - c) / (2i) = -i (z - c) / 2
        b.x = (T)0.5 * (zi - ci) * s;
        b.y = -(T)0.5 * (zr - cr) * s;
        reinterpret_cast<C2*>(ta)[idx] = a;
        if (tb) reinterpret_cast<C2*>(tb)[idx] = b;
    }
}

hipError_t launch_unpack_tables(const void* zre, const void* zim, void* ta, void* tb, int nx, int ny, int m, bool dbl,
                                hipStream_t s) {
    if (dbl)
        hipLaunchKernelGGL(unpack_tables_kernel<double>, dim3(2048), dim3(256), 0, s, (const double*)zre,
                           (const double*)zim, ta, tb, nx, ny, m);
    else
        hipLaunchKernelGGL(unpack_tables_kernel<float>, dim3(2048), dim3(256), 0, s, (const float*)zre,
                           (const float*)zim, ta, tb, nx, ny, m);
    return hipGetLastError();
}

// acc[k] (+)= s * ( G_a^[k] conj(Ta[k]) + G_b^[k] conj(Tb[k]) ), with G_a^, G_b^ unpacked from
// the spectrum Z^ = G_a^ + i G_b^ of a packed pair (tb may be null: single field, G_b^ = 0).
template <typename T>
__global__ void accumulate_pair_kernel(const T* zre, const T* zim, const void* ta, const void* tb, T* accre,
                                       T* accim, int nx, int ny, int m, T scale, int first) {
    using C2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
    const long long n = (long long)nx * ny * m;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int kx = (int)(idx % nx);
        const int ky = (int)((idx / nx) % ny);
        const int kt = (int)(idx / ((long long)nx * ny));
        const long long midx = ((long long)((m - kt) % m) * ny + (ny - ky) % ny) * nx + (nx - kx) % nx;
        const T zr = zre[idx], zi = zim[idx];
        const T cr = zre[midx], ci = -zim[midx];
        // G_a = (z + c)/2, G_b = (z - c)/(2i)
        const T ar = (T)0.5 * (zr + cr), ai = (T)0.5 * (zi + ci);
        const T br = (T)0.5 * (zi - ci), bi = -(T)0.5 * (zr - cr);
        const C2 wa = reinterpret_cast<const C2*>(ta)[idx];
        // G_a conj(Ta)
        T re = ar * wa.x + ai * wa.y;
        T im = ai * wa.x - ar * wa.y;
        if (tb) {
            const C2 wb = reinterpret_cast<const C2*>(tb)[idx];
            re += br * wb.x + bi * wb.y;
            im += bi * wb.x - br * wb.y;
        }
        re *= scale;
        im *= scale;
        if (first) {
            accre[idx] = re;
            accim[idx] = im;
        } else {
            accre[idx] += re;
            accim[idx] += im;
        }
    }
}

hipError_t launch_accumulate_pair(const void* zre, const void* zim, const void* ta, const void* tb, void* accre,
                                  void* accim, int nx, int ny, int m, double scale, int first, bool dbl,
                                  hipStream_t s) {
    if (dbl)
        hipLaunchKernelGGL(accumulate_pair_kernel<double>, dim3(2048), dim3(256), 0, s, (const double*)zre,
                           (const double*)zim, ta, tb, (double*)accre, (double*)accim, nx, ny, m, scale, first);
    else
        hipLaunchKernelGGL(accumulate_pair_kernel<float>, dim3(2048), dim3(256), 0, s, (const float*)zre,
                           (const float*)zim, ta, tb, (float*)accre, (float*)accim, nx, ny, m, (float)scale, first);
    return hipGetLastError();
}

// basis[q][j][i] = sum_images max(0, 1 - |r/h - q|), h = r_max/(n_knots-1)
__global__ void profile_basis_kernel(double* basis, int n_knots, double r_max, int nx, int ny) {
    const long long npts = (long long)nx * ny;
    const double h = r_max / (double)(n_knots - 1);
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < npts * n_knots;
         idx += (long long)gridDim.x * blockDim.x) {
        const int q = (int)(idx / npts);
        const long long p = idx - (long long)q * npts;
        const int i = (int)(p % nx), j = (int)(p / nx);
        const double x = -0.5 + (double)i / nx, y = -0.5 + (double)j / ny;
        double acc = 0.0;
        for (int a = -SE2C_PROFILE_IMAGES; a <= SE2C_PROFILE_IMAGES; ++a) {
            for (int b = -SE2C_PROFILE_IMAGES; b <= SE2C_PROFILE_IMAGES; ++b) {
                const double dx = x + a, dy = y + b;
                const double w = 1.0 - fabs(sqrt(dx * dx + dy * dy) / h - (double)q);
                if (w > 0.0) acc += w;
            }
        }
        basis[idx] = acc;
    }
}

// G[l][j][i] = sum_b g_b[l][j][i]  (FP64 accumulation, fixed order)
template <typename T>
__global__ void batch_sum_kernel(const T* g, double* out, long long n, int batch) {
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int b = 0; b < batch; ++b) acc += (double)g[(long long)b * n + idx];
        out[idx] = acc;
    }
}

// grad[q][l] = sum_p basis[q][p] G[l][p]; one block per (q, l), tree reduction.
__global__ void profile_contract_kernel(const double* basis, const double* G, double* grad, int n_knots, int m,
                                        long long npts) {
    __shared__ double red[256];
    const int q = blockIdx.x % n_knots;
    const int l = blockIdx.x / n_knots;
    const double* bq = basis + (long long)q * npts;
    const double* gl = G + (long long)l * npts;
    double acc = 0.0;
    for (long long p = threadIdx.x; p < npts; p += blockDim.x) acc += bq[p] * gl[p];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[(long long)q * m + l] = red[0];
}

hipError_t launch_profile_grad(const void* g, int batch, bool dbl, int n_knots, double r_max, int nx, int ny, int m,
                               double* basis, double* G, double* grad, hipStream_t s) {
    const long long npts = (long long)nx * ny;
    const long long n = npts * m;
    hipLaunchKernelGGL(profile_basis_kernel, dim3(2048), dim3(256), 0, s, basis, n_knots, r_max, nx, ny);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (dbl)
        hipLaunchKernelGGL(batch_sum_kernel<double>, dim3(2048), dim3(256), 0, s, (const double*)g, G, n, batch);
    else
        hipLaunchKernelGGL(batch_sum_kernel<float>, dim3(2048), dim3(256), 0, s, (const float*)g, G, n, batch);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(profile_contract_kernel, dim3(n_knots * m), dim3(256), 0, s, basis, G, grad, n_knots, m, npts);
    return hipGetLastError();
}

}  // namespace se2c
