// FP64 generation of twiddle tables and kernel coefficient tables on the GPU.
//
// Kernel coefficients are the finite Fourier coefficients of the sampled kernel
// (paper Sec. 4.1, eq. (FkLv)): rho^[k; L] = (-1)^{k1+k2} P^[k] / (Lx Ly Lr),
// where P^ is the DFT (Sec. 2.3, eq. (3DFT)) of the periodized kernel samples on
// Omega_L (eq. (OmL)).  A chain rho_1 * ... * rho_q uses the product of the
// tables (Thm. f*gP(2); Sec. 6.3); the product is formed here in FP64 and
// rounded once.
//
// A Gaussian x von Mises kernel exp(-|x|^2/2s^2) exp(k cos(theta - theta0)) is a
// product of 1-D factors in x, y and theta, and so is its lattice periodization;
// its table is the outer product Tx (x) Ty (x) Tt of three 1-D FFC vectors, each
// computed by a direct FP64 DFT with exactly reduced arguments ((k i) mod L).
#include <hip/hip_runtime.h>
#include <math.h>

#include "coeffs.hpp"
#include "fft_device.hpp"

namespace se2c {

// ------------------------------------------------------------------ twiddles
__global__ void twiddle_kernel(double2* out64, float2* out32, int L) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < L; j += gridDim.x * blockDim.x) {
        // exp(-2 pi i j / L) with the angle reduced exactly to the first quarter turn in
        // integers: quadrant q = floor(4j / L), remainder r = 4j - q L, so that
        // 2 pi j / L = q (pi/2) + (pi/2) r / L; sincospi takes the reduced angle and the
        // quadrant is an exact rotation by q quarter turns (the quarter-turn points come
        // out exact: r = 0 gives cos = 1, sin = 0).
        const long long j4 = 4LL * j;
        const int q = (int)(j4 / L);
        const long long r = j4 - (long long)q * L;
        double sr, cr;
        sincospi(0.5 * (double)r / (double)L, &sr, &cr);
        double c, s;
        switch (q & 3) {
            case 0: c = cr; s = sr; break;
            case 1: c = -sr; s = cr; break;
            case 2: c = -cr; s = -sr; break;
            default: c = sr; s = -cr; break;
        }
        double2 w;
        w.x = c;
        w.y = -s;
        if (out64) out64[j] = w;
        if (out32) out32[j] = make_float2((float)c, (float)(-s));
    }
}

hipError_t launch_twiddles(double2* out64, float2* out32, int L, hipStream_t s) {
    const int nthr = 256;
    const int nb = (L + nthr - 1) / nthr;
    hipLaunchKernelGGL(twiddle_kernel, dim3(nb), dim3(nthr), 0, s, out64, out32, L);
    return hipGetLastError();
}

// ------------------------------------------------- separable (Gauss x vM) tables
// One block per axis (blockIdx.x: 0 = x, 1 = y, 2 = theta).  acc64 holds the
// running FP64 product for the chain: [nx + ny + m] double2.
__device__ double periodized_gauss(double x, double sigma) {
    double acc = 0.0;
    for (int l = -SE2C_GAUSS_IMAGES; l <= SE2C_GAUSS_IMAGES; ++l) {
        const double d = x + (double)l;
        acc += exp(-(d * d) / (2.0 * sigma * sigma));
    }
    return acc;
}

__global__ void sep_factor_kernel(SepKernelParams kp, int nx, int ny, int m, double2* acc64, int first) {
    extern __shared__ double g[];  // samples (L doubles) then partial sums
    const int axis = blockIdx.x;
    const int L = axis == 0 ? nx : (axis == 1 ? ny : m);
    const int off = axis == 0 ? 0 : (axis == 1 ? nx : nx + ny);
    const int tid = threadIdx.x, nthr = blockDim.x;
    double* red = g + L;

    // 1) samples of the 1-D factor on Omega_L
    for (int i = tid; i < L; i += nthr) {
        if (axis < 2) {
            const double x = -0.5 + (double)i / (double)L;
            g[i] = periodized_gauss(x, kp.sigma);
        } else {
            const double t = 2.0 * M_PI * (double)i / (double)L;
            g[i] = exp(kp.kappa * (cos(t - kp.theta0) - 1.0));
        }
    }
    __syncthreads();
    // 2) sum of samples (for the discrete-mass normalisation)
    double part = 0.0;
    for (int i = tid; i < L; i += nthr) part += g[i];
    red[tid] = part;
    __syncthreads();
    for (int w = nthr / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    const double sum = red[0];

    // normalisation of this 1-D factor
    double norm;
    if (kp.norm == 0) {
        norm = 1.0 / sum;  // factor value 1 at k = 0: grid mean of the product is 1
    } else if (kp.norm == 1) {
        // continuous Haar mass: spatial factor 1/(sqrt(2 pi) sigma) per axis, angular
        // factor 1/I0(kappa) (the samples carry e^{-kappa}, matched by kp.ive0).
        norm = (axis < 2) ? 1.0 / ((double)L * sqrt(2.0 * M_PI) * kp.sigma)
                          : 1.0 / ((double)L * kp.ive0);
    } else {
        norm = (axis < 2) ? 1.0 / (double)L : exp(kp.kappa) / (double)L;
    }

    // 3) direct DFT with reduced arguments, sign (-1)^k on spatial axes, product
    for (int k = tid; k < L; k += nthr) {
        double re = 0.0, im = 0.0;
        for (int i = 0; i < L; ++i) {
            const long long r = ((long long)k * i) % L;
            double s, c;
            sincospi(2.0 * (double)r / (double)L, &s, &c);
            re += g[i] * c;
            im -= g[i] * s;
        }
        double sg = 1.0;
        if (axis < 2 && (signed_freq(k, L) & 1)) sg = -1.0;  // (-1)^k of the signed frequency
        re *= sg * norm;
        im *= sg * norm;
        double2 v;
        if (first) {
            v.x = re;
            v.y = im;
        } else {
            const double2 a = acc64[off + k];
            v.x = a.x * re - a.y * im;
            v.y = a.x * im + a.y * re;
        }
        acc64[off + k] = v;
    }
}

hipError_t launch_sep_factor(const SepKernelParams& kp, int nx, int ny, int m, double2* acc64, int first,
                             hipStream_t s) {
    const int nthr = 256;
    const int Lmax = nx > ny ? (nx > m ? nx : m) : (ny > m ? ny : m);
    const size_t lds = sizeof(double) * (size_t)(Lmax + nthr);
    hipLaunchKernelGGL(sep_factor_kernel, dim3(3), dim3(nthr), lds, s, kp, nx, ny, m, acc64, first);
    return hipGetLastError();
}

// ---------------------------------------------------------- full 3-D tables
// spec = (re, im) planes of the FP64 DFT of the samples.  Multiplies the FFC
// (-1)^{k1+k2} P^[k] / norm into acc (complex FP64 [m][ny][nx]).  norm is the
// sample sum (discrete normalisation, = P^[0]) or n.
__global__ void full_fold_kernel(const double* re, const double* im, double2* acc, long long n, int nx, int ny,
                                 int norm_mode, int first) {
    const double norm = norm_mode == 0 ? re[0] : (double)n;
    const double inv = 1.0 / norm;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int kx = (int)(i % nx);
        const int ky = (int)((i / nx) % ny);
        const double sg = ((signed_freq(kx, nx) + signed_freq(ky, ny)) & 1) ? -inv : inv;
        double2 v;
        v.x = re[i] * sg;
        v.y = im[i] * sg;
        if (!first) {
            const double2 a = acc[i];
            double2 w;
            w.x = a.x * v.x - a.y * v.y;
            w.y = a.x * v.y + a.y * v.x;
            v = w;
        }
        acc[i] = v;
    }
}

// Multiply a separable FP64 factor triple (acc64 layout [nx | ny | m]) into a full table.
__global__ void full_fold_sep_kernel(const double2* sep, double2* acc, long long n, int nx, int ny, int first) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int kx = (int)(i % nx);
        const int ky = (int)((i / nx) % ny);
        const int kt = (int)(i / ((long long)nx * ny));
        double2 ab;
        const double2 fx = sep[kx];
        const double2 fy = sep[nx + ky];
        const double2 ft = sep[nx + ny + kt];
        ab.x = fx.x * fy.x - fx.y * fy.y;
        ab.y = fx.x * fy.y + fx.y * fy.x;
        double2 v;
        v.x = ab.x * ft.x - ab.y * ft.y;
        v.y = ab.x * ft.y + ab.y * ft.x;
        if (!first) {
            const double2 p = acc[i];
            double2 w;
            w.x = p.x * v.x - p.y * v.y;
            w.y = p.x * v.y + p.y * v.x;
            v = w;
        }
        acc[i] = v;
    }
}

hipError_t launch_full_fold(const double* re, const double* im, double2* acc, long long n, int nx, int ny,
                            int norm_mode, int first, hipStream_t s) {
    hipLaunchKernelGGL(full_fold_kernel, dim3(1024), dim3(256), 0, s, re, im, acc, n, nx, ny, norm_mode, first);
    return hipGetLastError();
}

hipError_t launch_full_fold_sep(const double2* sep, double2* acc, long long n, int nx, int ny, int first,
                                hipStream_t s) {
    hipLaunchKernelGGL(full_fold_sep_kernel, dim3(1024), dim3(256), 0, s, sep, acc, n, nx, ny, first);
    return hipGetLastError();
}

// Round an FP64 complex array into the table dtype.
__global__ void round_kernel(const double2* src, void* dst, long long n, int dbl) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        if (dbl) {
            reinterpret_cast<double2*>(dst)[i] = src[i];
        } else {
            reinterpret_cast<float2*>(dst)[i] = make_float2((float)src[i].x, (float)src[i].y);
        }
    }
}

hipError_t launch_round(const double2* src, void* dst, long long n, int dbl, hipStream_t s) {
    long long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(round_kernel, dim3((unsigned)nb), dim3(256), 0, s, src, dst, n, dbl);
    return hipGetLastError();
}

// Quarter table of a FULL table T[m][ny][nx] (complex, float2 or double2):
// q[k3][b][a] = T[k3][b][a] for 0 <= a <= nx/2, 0 <= b <= ny/2, and the statistics of the
// reflection symmetry max_k |T[k3][k2][k1] - T[k3][|k2|][|k1|]| (|k| = min(k, L - k), the
// nonnegative signed frequency) and max_k |T[k]|, FP64, as the bit patterns of nonnegative
// doubles (which order like the values) under atomicMax: stats[0], stats[1].
template <typename CT>
__global__ void quarter_kernel(const CT* __restrict__ full, CT* __restrict__ q, int nx, int ny, int m,
                               unsigned long long* stats) {
    const int hx = nx / 2 + 1, hy = ny / 2 + 1;
    const long long n = (long long)nx * ny * m;
    double dev = 0.0, big = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int kx = (int)(i % nx);
        const long long r = i / nx;
        const int ky = (int)(r % ny);
        const int kt = (int)(r / ny);
        const int ax = min(kx, nx - kx), ay = min(ky, ny - ky);
        const CT v = full[i];
        const CT w = full[((long long)kt * ny + ay) * nx + ax];
        dev = fmax(dev, hypot((double)v.x - (double)w.x, (double)v.y - (double)w.y));
        big = fmax(big, hypot((double)v.x, (double)v.y));
        if (kx == ax && ky == ay) q[((long long)kt * hy + ay) * hx + ax] = v;
    }
    for (int o = 32; o > 0; o >>= 1) {
        dev = fmax(dev, __shfl_xor(dev, o));
        big = fmax(big, __shfl_xor(big, o));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&stats[0], (unsigned long long)__double_as_longlong(dev));
        atomicMax(&stats[1], (unsigned long long)__double_as_longlong(big));
    }
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

hipError_t launch_quarter(const void* full, void* q, int nx, int ny, int m, int dbl, unsigned long long* stats,
                          hipStream_t s) {
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, stats, 2);
    const long long n = (long long)nx * ny * m;
    long long nb = (n + 255) / 256;
    if (nb > 8192) nb = 8192;
    if (dbl)
        hipLaunchKernelGGL(quarter_kernel<double2>, dim3((unsigned)nb), dim3(256), 0, s,
                           reinterpret_cast<const double2*>(full), reinterpret_cast<double2*>(q), nx, ny, m, stats);
    else
        hipLaunchKernelGGL(quarter_kernel<float2>, dim3((unsigned)nb), dim3(256), 0, s,
                           reinterpret_cast<const float2*>(full), reinterpret_cast<float2*>(q), nx, ny, m, stats);
    return hipGetLastError();
}

// One weighted term of a sum of kernel tables, accumulated in FP64.
__global__ void axpy64_kernel(const double2* __restrict__ x, double2* __restrict__ y, long long n, double w,
                              int first) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const double2 v = x[i];
        double2 acc = first ? make_double2(0.0, 0.0) : y[i];
        acc.x = fma(w, v.x, acc.x);
        acc.y = fma(w, v.y, acc.y);
        y[i] = acc;
    }
}

hipError_t launch_axpy64(const double2* x, double2* y, long long n, double w, int first, hipStream_t s) {
    const int nthr = 256;
    const long long want = (n + nthr - 1) / nthr;
    const int nb = (int)(want < 16384 ? want : 16384);
    hipLaunchKernelGGL(axpy64_kernel, dim3(nb), dim3(nthr), 0, s, x, y, n, w, first);
    return hipGetLastError();
}

// Radial-profile kernel samples (FP64):
// P[l][j][i] = sum_images sum_q prof[q][l] * hat_q(|x_ij + image|),
// hat_q(r) = max(0, 1 - |r/h - q|), h = r_max/(n_knots-1).
// P[l][j][i] = sum over lattice images of the hat interpolant of prof[.][l] at
// r = |x_ij + image|.  One thread per (point, 16 consecutive theta samples): the
// radius and its knot interval are computed once per image and reused for the 16 l.
constexpr int kProfileLChunk = 16;

__global__ void profile_samples_kernel(const double* prof, int n_knots, double r_max, int nx, int ny, int m,
                                       double* out) {
    const long long npts = (long long)nx * ny;
    const int nlc = (m + kProfileLChunk - 1) / kProfileLChunk;
    const double h = r_max / (double)(n_knots - 1);
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < npts * nlc;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long p = idx % npts;
        const int l0 = (int)(idx / npts) * kProfileLChunk;
        const int nl = m - l0 < kProfileLChunk ? m - l0 : kProfileLChunk;
        const int i = (int)(p % nx), j = (int)(p / nx);
        const double x = -0.5 + (double)i / nx, y = -0.5 + (double)j / ny;
        double acc[kProfileLChunk];
#pragma unroll
        for (int c = 0; c < kProfileLChunk; ++c) acc[c] = 0.0;
        for (int a = -SE2C_PROFILE_IMAGES; a <= SE2C_PROFILE_IMAGES; ++a) {
            for (int b = -SE2C_PROFILE_IMAGES; b <= SE2C_PROFILE_IMAGES; ++b) {
                const double dx = x + a, dy = y + b;
                const double u = sqrt(dx * dx + dy * dy) / h;
                const int q0 = (int)floor(u);
                if (q0 >= n_knots) continue;
                const double t = u - q0;
                const double* p0 = prof + (long long)q0 * m + l0;
                const bool has1 = q0 + 1 < n_knots;
#pragma unroll
                for (int c = 0; c < kProfileLChunk; ++c) {
                    if (c < nl) {
                        acc[c] += (1.0 - t) * p0[c];
                        if (has1) acc[c] += t * p0[m + c];
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < kProfileLChunk; ++c)
            if (c < nl) out[(long long)(l0 + c) * npts + p] = acc[c];
    }
}

// Exponential-coordinates Gaussian exp(-((t/2)/sin(t/2))^2 |x + l|^2 / (2 sigma^2) - t^2 / (2 sigma^2)),
// summed over lattice images l, with theta_l wrapped to (-pi, pi] (principal logarithm of
// SE(2)).  One thread per grid point.
__global__ void exp_gauss_samples_kernel(double sigma, int nx, int ny, int m, double* out) {
    const long long n = (long long)nx * ny * m;
    const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(idx % nx);
        const int j = (int)((idx / nx) % ny);
        const int l = (int)(idx / ((long long)nx * ny));
        double t = 2.0 * M_PI * (double)l / (double)m;
        if (t > M_PI) t -= 2.0 * M_PI;
        const double h = 0.5 * t;
        const double fac = (h == 0.0) ? 1.0 : h / sin(h);
        const double x = -0.5 + (double)i / nx, y = -0.5 + (double)j / ny;
        double acc = 0.0;
        for (int a = -SE2C_GAUSS_IMAGES; a <= SE2C_GAUSS_IMAGES; ++a) {
            for (int b = -SE2C_GAUSS_IMAGES; b <= SE2C_GAUSS_IMAGES; ++b) {
                const double dx = x + a, dy = y + b;
                acc += exp(-fac * fac * (dx * dx + dy * dy) * inv2s2);
            }
        }
        out[idx] = acc * exp(-t * t * inv2s2);
    }
}

hipError_t launch_exp_gauss_samples(double sigma, int nx, int ny, int m, double* out, hipStream_t s) {
    hipLaunchKernelGGL(exp_gauss_samples_kernel, dim3(2048), dim3(256), 0, s, sigma, nx, ny, m, out);
    return hipGetLastError();
}

// ------------------------------------- radial-profile tables from the basis spectrum
// The samples of a radial profile are P[l] = sum_q prof[q][l] H_q with H_q the periodized
// hat basis on the spatial grid, so their 3-D DFT (eq. (3DFT)) is
//     P^[k3][k2][k1] = sum_q prof^[k3][q] H_q^[k2][k1],
// prof^ the DFT of prof along theta and H_q^ the 2-D DFT of H_q (built once per geometry).
// H_q is real, periodic and even in x and in y (H[j][N - i] = H[j][i], the grid point
// x_{N-i} being -x_i mod 1), so H_q^ is real and even in k1 and in k2: only the quadrant
// 0 <= k1 <= Nx/2, 0 <= k2 <= Ny/2 is kept, as real numbers.  The FFC table is then
// (-1)^{k1+k2} P^ / norm (eq. (FkLv)), all in FP64.

// X[q][j][k1] = sum_i H[q][j][i] w_nx^{k1 i}, k1 <= nx/2
__global__ void basis_dft_x_kernel(const double* basis, const double2* twx, int nq, int nx, int ny, double2* out) {
    const int hx = nx / 2 + 1;
    const long long total = (long long)nq * ny * hx;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const int k1 = (int)(idx % hx);
        const long long row = idx / hx;  // q * ny + j
        const double* h = basis + row * nx;
        double re = 0.0, im = 0.0;
        int t = 0;
        for (int i = 0; i < nx; ++i) {
            const double2 w = twx[t];
            re += h[i] * w.x;
            im += h[i] * w.y;
            t += k1;
            if (t >= nx) t -= nx;
        }
        out[idx] = make_double2(re, im);
    }
}

// hr[q][k2][k1] = Re sum_j X[q][j][k1] w_ny^{k2 j}, k1 <= nx/2, k2 <= ny/2 (the imaginary
// part vanishes by the symmetry above)
__global__ void basis_dft_y_kernel(const double2* X, const double2* twy, int nq, int nx, int ny, double* out) {
    const int hx = nx / 2 + 1, hy = ny / 2 + 1;
    const long long quad = (long long)hx * hy;
    const long long total = (long long)nq * quad;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const int q = (int)(idx / quad);
        const long long rem = idx - (long long)q * quad;
        const int k2 = (int)(rem / hx), k1 = (int)(rem % hx);
        const double2* x = X + (long long)q * ny * hx + k1;
        double re = 0.0;
        int t = 0;
        for (int j = 0; j < ny; ++j) {
            const double2 v = x[(long long)j * hx];
            const double2 w = twy[t];
            re += v.x * w.x - v.y * w.y;
            t += k2;
            if (t >= ny) t -= ny;
        }
        out[idx] = re;
    }
}

// phT[g][q][i] = prof^[k3 = g + 4 i][q] = sum_l prof[q][l] w_m^{k3 l} (zero for k3 >= m):
// the values one wave of the fold kernel needs for knot q, contiguous
__global__ void profile_theta_dft_kernel(const double* prof, const double2* twm, int nq, int m, double2* pht) {
    constexpr int KI = kProfileFoldMaxM / 4;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < 4 * nq * KI; idx += gridDim.x * blockDim.x) {
        const int i = idx % KI;
        const int q = (idx / KI) % nq;
        const int g = idx / (KI * nq);
        const int k3 = g + 4 * i;
        double re = 0.0, im = 0.0;
        if (k3 < m) {
            int t = 0;
            for (int l = 0; l < m; ++l) {
                const double v = prof[(long long)q * m + l];
                re += v * twm[t].x;
                im += v * twm[t].y;
                t += k3;
                if (t >= m) t -= m;
            }
        }
        pht[idx] = make_double2(re, im);
    }
}

// acc[k3][k2][k1] (*)= (-1)^{k1+k2} / norm * sum_q prof^[k3][q] hr[q][|k2|][|k1|], norm = P^[0]
// (the sample sum, discrete mass) or n.  One lane per quadrant frequency (|k1|, |k2|); the
// four waves of a block and the four blocks along y split k3 (wave g of block y:
// k3 = g + 4 (4 y + i), i < 4), each lane keeping 4 complex sums while hr[q] streams through
// (four blocks per 64 frequencies: a quarter of the sums per lane measured faster than one
// block holding 16); the wave-uniform prof^ values come through scalar loads.  Each result
// goes to the up to four mirrored frequencies.  Requires m, n_knots <= 64.
__global__ void __launch_bounds__(256) profile_fold_kernel(const double* hr, const double2* pht, int nq, int nx,
                                                           int ny, int m, int norm_mode, double2* acc, int first) {
    constexpr int KT = kProfileFoldMaxM / 4;  // k3 values per wave over the whole grid
    constexpr int KI = KT / 4;                // of them in this block (blockIdx.y picks the quarter)
    const int hx = nx / 2 + 1, hy = ny / 2 + 1;
    const long long quad = (long long)hx * hy;
    const long long nxy = (long long)nx * ny;
    const int g = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long kq0 = (long long)blockIdx.x * 64 + (threadIdx.x & 63);
    const long long kq = kq0 < quad ? kq0 : quad - 1;  // clamped lanes compute, never store
    double2 sum[KI];
#pragma unroll
    for (int i = 0; i < KI; ++i) sum[i] = make_double2(0.0, 0.0);
    const double2* pw = pht + (long long)g * nq * KT + blockIdx.y * KI;
    double h = hr[kq];
    for (int q = 0; q < nq; ++q) {
        const double hn = hr[(long long)(q + 1 < nq ? q + 1 : q) * quad + kq];
#pragma unroll
        for (int i = 0; i < KI; ++i) {
            const double2 a = pw[q * KT + i];
            sum[i].x += a.x * h;
            sum[i].y += a.y * h;
        }
        h = hn;
    }
    if (kq0 >= quad) return;
    double inv = 1.0 / (double)(nxy * m);
    if (norm_mode == 0) {
        double s0 = 0.0;  // P^[0,0,0]: the sum of the (real) samples
        for (int q = 0; q < nq; ++q) s0 += pht[(long long)q * KT].x * hr[(long long)q * quad];
        inv = 1.0 / s0;
    }
    const int a1 = (int)(kq % hx), a2 = (int)(kq / hx);
    const int m1 = (nx - a1) % nx, m2 = (ny - a2) % ny;  // mirrored indices
    const double sg = ((signed_freq(a1, nx) + signed_freq(a2, ny)) & 1) ? -inv : inv;
    const long long pos[4] = {(long long)a2 * nx + a1, (long long)a2 * nx + m1, (long long)m2 * nx + a1,
                              (long long)m2 * nx + m1};
    const bool use[4] = {true, m1 != a1, m2 != a2, m1 != a1 && m2 != a2};
#pragma unroll
    for (int i = 0; i < KI; ++i) {
        const int k3 = g + 4 * (blockIdx.y * KI + i);
        if (k3 < m) {
            const double2 v = make_double2(sum[i].x * sg, sum[i].y * sg);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (!use[c]) continue;
                const long long o = (long long)k3 * nxy + pos[c];
                double2 w = v;
                if (!first) {
                    const double2 b = acc[o];
                    w = make_double2(b.x * v.x - b.y * v.y, b.x * v.y + b.y * v.x);
                }
                acc[o] = w;
            }
        }
    }
}

hipError_t launch_basis_dft(const double* basis, const double2* twx, const double2* twy, int nq, int nx, int ny,
                            double2* tmp, double* hr, hipStream_t s) {
    hipLaunchKernelGGL(basis_dft_x_kernel, dim3(4096), dim3(256), 0, s, basis, twx, nq, nx, ny, tmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(basis_dft_y_kernel, dim3(4096), dim3(256), 0, s, tmp, twy, nq, nx, ny, hr);
    return hipGetLastError();
}

hipError_t launch_profile_fold(const double* prof, const double2* twm, const double* hr, int nq, int nx, int ny,
                               int m, int norm_mode, double2* pht, double2* acc, int first, hipStream_t s) {
    const int np = 4 * nq * (kProfileFoldMaxM / 4);
    hipLaunchKernelGGL(profile_theta_dft_kernel, dim3((np + 255) / 256), dim3(256), 0, s, prof, twm, nq, m, pht);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long quad = (long long)(nx / 2 + 1) * (ny / 2 + 1);
    hipLaunchKernelGGL(profile_fold_kernel, dim3((unsigned)((quad + 63) / 64), 4), dim3(256), 0, s, hr, pht, nq, nx, ny,
                       m, norm_mode, acc, first);
    return hipGetLastError();
}

hipError_t launch_profile_samples(const double* prof, int n_knots, double r_max, int nx, int ny, int m, double* out,
                                  hipStream_t s) {
    hipLaunchKernelGGL(profile_samples_kernel, dim3(2048), dim3(256), 0, s, prof, n_knots, r_max, nx, ny, m, out);
    return hipGetLastError();
}

}  // namespace se2c
