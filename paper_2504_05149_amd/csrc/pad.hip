// Zero-padded spectrum for evaluating S_K on a finer grid (paper Sec. 4.1 eq.
// (MatSKfonG), Sec. 6.1 eq. (MatSKfgonG), Prop. LtoN1D).
//
// The product spectrum H of one field pair lives on the sampling grid L = (Lx, Ly, Lm)
// as two real planes (re, im), layout [k3][k2][k1].  The spectrum on the finer grid
// G >= L keeps every signed frequency k of the L-grid at its G-grid index tau_G(k)
// and is zero elsewhere.  For even L the index L/2 holds the frequencies +-L/2
// together; on a finer grid it is split in halves between tau_G(-L/2) and
// tau_G(+L/2), so that the evaluation of a real field stays real (when G = L both are
// the same index and the value is kept whole).  One thread per G-grid element of every
// pair; every element of the G-spectra is written.  Pair i reads its two L planes at
// src + i src_stride (re, then im n_L later) and writes its two G planes at
// dst + i dst_stride (re, then im n_G later; the last pair's im plane goes to `lone` when
// that is given: a field without a partner).
#include <hip/hip_runtime.h>

#include "fft_device.hpp"
#include "passes.hpp"

namespace se2c {

template <typename T>
__global__ void pad_spectrum_kernel(const T* __restrict__ src, T* __restrict__ dst, T* __restrict__ lone, int nitems,
                                    long long src_stride, long long dst_stride, int lx, int ly, int lm, int gx,
                                    int gy, int gm) {
    const long long ng = (long long)gx * gy * gm;
    const long long nl = (long long)lx * ly * lm;
    const long long total = ng * nitems;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int item = (int)(i / ng);
        const long long e = i - (long long)item * ng;
        const int g1 = (int)(e % gx);
        const int g2 = (int)((e / gx) % gy);
        const int g3 = (int)(e / ((long long)gx * gy));
        bool h1, h2, h3;
        const int s1 = pad_source(g1, gx, lx, &h1);
        const int s2 = pad_source(g2, gy, ly, &h2);
        const int s3 = pad_source(g3, gm, lm, &h3);
        T re = (T)0, im = (T)0;
        if (s1 >= 0 && s2 >= 0 && s3 >= 0) {
            const T* sre = src + (long long)item * src_stride;
            const long long o = ((long long)s3 * ly + s2) * lx + s1;
            T w = (T)1;
            if (h1) w *= (T)0.5;
            if (h2) w *= (T)0.5;
            if (h3) w *= (T)0.5;
            re = w * sre[o];
            im = w * sre[nl + o];
        }
        T* dre = dst + (long long)item * dst_stride;
        T* dim = (lone && item == nitems - 1) ? lone : dre + ng;
        dre[e] = re;
        dim[e] = im;
    }
}

hipError_t launch_pad_spectrum(const void* src, void* dst, void* lone, int nitems, long long src_stride,
                               long long dst_stride, int lx, int ly, int lm, int gx, int gy, int gm, bool dbl,
                               hipStream_t s) {
    const long long total = (long long)gx * gy * gm * nitems;
    const int nthr = 256;
    const long long want = (total + nthr - 1) / nthr;
    const int nb = (int)(want < 16384 ? want : 16384);
    if (dbl)
        hipLaunchKernelGGL(pad_spectrum_kernel<double>, dim3(nb), dim3(nthr), 0, s, (const double*)src, (double*)dst,
                           (double*)lone, nitems, src_stride, dst_stride, lx, ly, lm, gx, gy, gm);
    else
        hipLaunchKernelGGL(pad_spectrum_kernel<float>, dim3(nb), dim3(nthr), 0, s, (const float*)src, (float*)dst,
                           (float*)lone, nitems, src_stride, dst_stride, lx, ly, lm, gx, gy, gm);
    return hipGetLastError();
}

}  // namespace se2c
