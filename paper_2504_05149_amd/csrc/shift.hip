// Translation-phase tables for kernels that are sums of SE(2)-shifts of one kernel rho
// radial in translations (the outlook of Sec. 1: f2 ~ sum_k a_k rho_k).
//
// With rho_k(g) = rho(s_k^{-1} o g), s_k = (t_k, R_phi_k) (group law eq. (SE2law)),
// radiality of rho turns rho_k(h^{-1} o g) for h = (y, alpha), g = (x, theta) into
// rho(x - y - R_alpha t_k, theta - alpha - phi_k): convolving with rho_k is convolving
// with rho (Thm. f*gP: a product of coefficients) after translating every theta-slice
// alpha of f by R_alpha t_k and shifting the field by phi_k in theta.  On the spatial
// finite Fourier coefficients of a slice the translation is the phase
//   e^{-2 pi i (k1, k2) . R_alpha t_k}
// (for an even length the Nyquist index holds +-L/2 in halves: the phase there is the
// real cos(pi L tau)).  Terms with the same theta shift (a roll by r grid angles) share
// one table, the weighted sum of their phases.
#include "fft_device.hpp"
#include "shift.hpp"

namespace se2c {

// e^{-2 pi i k tau} for signed frequency k of index t (cos(pi L tau) at an even length's
// Nyquist index), with k tau reduced to [-1/2, 1/2] before the angle is formed.
__device__ __forceinline__ double2 axis_phase(int t, int L, double tau) {
    if (!(L & 1) && 2 * t == L) return make_double2(cospi((double)L * tau), 0.0);
    const int k = t <= (L - 1) / 2 ? t : t - L;
    const double x = (double)k * tau;
    const double r = x - rint(x);
    double s, c;
    sincospi(-2.0 * r, &s, &c);
    return make_double2(c, s);
}

__global__ void shift_table_kernel(ShiftClassArgs a, void* out, int dbl) {
    const long long n = (long long)a.nx * a.ny * a.m;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t1 = (int)(i % a.nx);
    const int t2 = (int)((i / a.nx) % a.ny);
    const int al = (int)(i / ((long long)a.nx * a.ny));
    double sa, ca;
    sincospi(2.0 * (double)al / (double)a.m, &sa, &ca);
    double re = 0.0, im = 0.0;
    for (int k = 0; k < a.nterm; ++k) {
        const ShiftTerm& s = a.t[k];
        const double ux = ca * s.tx - sa * s.ty;  // R_alpha t
        const double uy = sa * s.tx + ca * s.ty;
        const double2 ex = axis_phase(t1, a.nx, ux);
        const double2 ey = axis_phase(t2, a.ny, uy);
        re += s.w * (ex.x * ey.x - ex.y * ey.y);
        im += s.w * (ex.x * ey.y + ex.y * ey.x);
    }
    if (dbl)
        reinterpret_cast<double2*>(out)[i] = make_double2(re, im);
    else
        reinterpret_cast<float2*>(out)[i] = make_float2((float)re, (float)im);
}

hipError_t launch_shift_table(const ShiftClassArgs& a, void* out, bool dbl, hipStream_t s) {
    const long long n = (long long)a.nx * a.ny * a.m;
    const int nt = 256;
    hipLaunchKernelGGL(shift_table_kernel, dim3((unsigned)((n + nt - 1) / nt)), dim3(nt), 0, s, a, out, dbl ? 1 : 0);
    return hipGetLastError();
}

}  // namespace se2c
