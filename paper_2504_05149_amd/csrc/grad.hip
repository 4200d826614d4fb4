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
//               sample expansion); FP64, deterministic (split-K partial products summed
//               in a fixed order, no atomics), on the matrix cores up to 64 knots and 64
//               angles.  The basis is built once per geometry.
#include <hip/hip_runtime.h>

#include "coeffs.hpp"
#include "fft_device.hpp"
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
        const T s = ((signed_freq(kx, nx) + signed_freq(ky, ny)) & 1) ? -inv : inv;
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

// part[s][q][l] = sum over points p of split s of basis[q][p] G[l][p]: one 64 x 64 output
// tile per block (4 x 4 per thread), points staged through LDS 32 at a time.
constexpr int kGemmTile = 64;
constexpr int kGemmK = 32;

__global__ void __launch_bounds__(256) profile_contract_partial_kernel(const double* basis, const double* G,
                                                                       double* part, int n_knots, int m,
                                                                       long long npts, int kchunk) {
    __shared__ double hs[kGemmTile][kGemmK + 1];
    __shared__ double gs[kGemmTile][kGemmK + 1];
    const int ntq = (n_knots + kGemmTile - 1) / kGemmTile;
    const int split = blockIdx.x;
    const int q0 = (blockIdx.y % ntq) * kGemmTile;
    const int l0 = (blockIdx.y / ntq) * kGemmTile;
    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;
    double acc[4][4] = {};
    const long long pbeg = (long long)split * kchunk;
    const long long pend = pbeg + kchunk < npts ? pbeg + kchunk : npts;
    for (long long p0 = pbeg; p0 < pend; p0 += kGemmK) {
        for (int e = tid; e < kGemmTile * kGemmK; e += 256) {
            const int r = e / kGemmK, c = e - r * kGemmK;
            const long long pp = p0 + c;
            const bool inp = pp < pend;
            hs[r][c] = (inp && q0 + r < n_knots) ? basis[(long long)(q0 + r) * npts + pp] : 0.0;
            gs[r][c] = (inp && l0 + r < m) ? G[(long long)(l0 + r) * npts + pp] : 0.0;
        }
        __syncthreads();
        for (int c = 0; c < kGemmK; ++c) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = hs[ty * 4 + i][c];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = gs[tx * 4 + j][c];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int q = q0 + ty * 4 + i;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int l = l0 + tx * 4 + j;
            if (q < n_knots && l < m) part[((long long)split * n_knots + q) * m + l] = acc[i][j];
        }
    }
}

// The same contraction on the matrix cores when n_knots <= 64 and m <= 64 (the common
// case: a 64 x 64 output, K = Nx Ny points): one block per kMfmaChunk points, wave w takes
// the knots 16 w .. 16 w + 15 against all 64 l as four 16 x 16 tiles of
// v_mfma_f64_16x16x4 (FP64 products and sums).  Operand layout of the instruction: lane
// (i = lane % 16, k = lane / 16) holds A[i][k] = basis[q0 + i][p + k] and B[k][j] with
// j = i, G[l0 + j][p + k]; the 16 x 16 result sits in lane (c = lane % 16) as rows
// lane / 16 + 4 r, r < 4 (checked on the device with a product of known factors).
// Operands come straight from global memory: each lane's row advances 4 points per step,
// so a row's cache lines are used whole over 8 steps.  Knots past n_knots, angles past m
// and points past the chunk read a clamped address and are zeroed.  At 256 x 256 x 64 with
// 64 knots: 51 us plus 6 us for the reduction of its 256 splits, against 46 + 17 us for the
// LDS-staged kernel above (bound by its LDS reads, 8 per 16 FMAs); point-major copies of
// the basis and G measured slower (86 us).
typedef double d4_t __attribute__((ext_vector_type(4)));
constexpr int kMfmaChunk = 256;

__global__ void __launch_bounds__(256) profile_contract_mfma_kernel(const double* basis, const double* G,
                                                                    double* part, int n_knots, int m,
                                                                    long long npts) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 15, kk = lane >> 4;
    const int q = 16 * w + i;
    const bool qok = q < n_knots;
    const double* arow = basis + (long long)(qok ? q : 0) * npts;
    const double* brow[4];
    bool lok[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int l = 16 * j + i;
        lok[j] = l < m;
        brow[j] = G + (long long)(lok[j] ? l : 0) * npts;
    }
    const long long pbeg = (long long)blockIdx.x * kMfmaChunk;
    const long long pend = pbeg + kMfmaChunk < npts ? pbeg + kMfmaChunk : npts;
    d4_t acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
    for (int st = 0; st < kMfmaChunk / 4; ++st) {  // a short last chunk runs on zeros
        const long long p = pbeg + 4 * st + kk;
        const bool pok = p < pend;
        const long long pc = pok ? p : pend - 1;
        const double av = arow[pc];
        const double a = (qok && pok) ? av : 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double bv = brow[j][pc];
            const double b = (lok[j] && pok) ? bv : 0.0;
            acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
        }
    }
    double* out = part + (long long)blockIdx.x * n_knots * m;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int l = 16 * j + i;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int qq = 16 * w + kk + 4 * r;
            if (qq < n_knots && l < m) out[(long long)qq * m + l] = acc[j][r];
        }
    }
}

// grad[o] = sum_s part[s][o] (o = q m + l): 16 outputs per block, split s summed by
// thread group s mod 16 in increasing order, then the 16 group sums in order
// (a fixed summation order: bitwise reproducible).
__global__ void __launch_bounds__(256) profile_contract_reduce_kernel(const double* part, double* grad, int nsplit,
                                                                      long long nout) {
    __shared__ double red[16][17];
    const int oi = threadIdx.x % 16, grp = threadIdx.x / 16;
    const long long o = (long long)blockIdx.x * 16 + oi;
    double acc = 0.0;
    if (o < nout)
        for (int sp = grp; sp < nsplit; sp += 16) acc += part[(long long)sp * nout + o];
    red[grp][oi] = acc;
    __syncthreads();
    if (grp == 0 && o < nout) {
        double t = 0.0;
        for (int gi = 0; gi < 16; ++gi) t += red[gi][oi];
        grad[o] = t;
    }
}

hipError_t launch_profile_basis(double* basis, int n_knots, double r_max, int nx, int ny, hipStream_t s) {
    hipLaunchKernelGGL(profile_basis_kernel, dim3(2048), dim3(256), 0, s, basis, n_knots, r_max, nx, ny);
    return hipGetLastError();
}

int profile_grad_splits(long long npts) { return (int)((npts + kProfileChunk - 1) / kProfileChunk); }

hipError_t launch_profile_grad(const void* g, int batch, bool dbl, int n_knots, int nx, int ny, int m,
                               const double* basis, double* G, double* part, double* grad, hipStream_t s) {
    const long long npts = (long long)nx * ny;
    const long long n = npts * m;
    if (dbl)
        hipLaunchKernelGGL(batch_sum_kernel<double>, dim3(2048), dim3(256), 0, s, (const double*)g, G, n, batch);
    else
        hipLaunchKernelGGL(batch_sum_kernel<float>, dim3(2048), dim3(256), 0, s, (const float*)g, G, n, batch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int nsplit;
    if (n_knots <= 64 && m <= 64) {
        // fewer splits than the workspace holds (kMfmaChunk >= kProfileChunk points each)
        nsplit = (int)((npts + kMfmaChunk - 1) / kMfmaChunk);
        hipLaunchKernelGGL(profile_contract_mfma_kernel, dim3(nsplit), dim3(256), 0, s, basis, G, part, n_knots, m,
                           npts);
    } else {
        nsplit = profile_grad_splits(npts);
        const int ntiles = ((n_knots + kGemmTile - 1) / kGemmTile) * ((m + kGemmTile - 1) / kGemmTile);
        hipLaunchKernelGGL(profile_contract_partial_kernel, dim3(nsplit, ntiles), dim3(256), 0, s, basis, G, part,
                           n_knots, m, npts, kProfileChunk);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long nout = (long long)n_knots * m;
    hipLaunchKernelGGL(profile_contract_reduce_kernel, dim3((unsigned)((nout + 15) / 16)), dim3(256), 0, s, part,
                       grad, nsplit, nout);
    return hipGetLastError();
}

}  // namespace se2c
