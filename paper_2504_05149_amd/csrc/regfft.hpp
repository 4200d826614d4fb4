// In-register DFT codelets with compile-time twiddles (FP32/FP64).
//
// dft_reg<N, INV>(v): natural-order in, natural-order out, v[0..N-1] held in
// registers (every index is a compile-time constant after unrolling).  N = 2, 4,
// 8, 16 use the hand-written butterflies of fft_device.hpp; N = 16 * B (B = 2, 4)
// is composed as B radix-16 DFTs on the stride-B subsequences, twiddles
// w_N^{b k1}, then 16 radix-B DFTs.  The codelet twiddles are evaluated at compile
// time in double (Taylor series on a quarter turn) and rounded to T.
#pragma once
#include <type_traits>

#include "fft_device.hpp"

namespace se2c {

constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double x) {
    double term = x, sum = x;
    for (int k = 1; k < 24; ++k) {
        term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double taylor_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 24; ++k) {
        term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}
// cos and sin of 2 pi j / N, reduced exactly to the first quarter turn.
constexpr double cos2pi(int j, int n) {
    j %= n;
    if (j < 0) j += n;
    const int q = (4 * j) / n;          // quadrant
    const int r = 4 * j - q * n;        // remainder in units of (pi/2)/n
    const double a = 0.5 * kPi * (double)r / (double)n;
    const double c = taylor_cos(a), s = taylor_sin(a);
    return q == 0 ? c : (q == 1 ? -s : (q == 2 ? -c : s));
}
constexpr double sin2pi(int j, int n) {
    j %= n;
    if (j < 0) j += n;
    const int q = (4 * j) / n;
    const int r = 4 * j - q * n;
    const double a = 0.5 * kPi * (double)r / (double)n;
    const double c = taylor_cos(a), s = taylor_sin(a);
    return q == 0 ? s : (q == 1 ? c : (q == 2 ? -s : -c));
}

// Compile-time loop: f(std::integral_constant<int, I>) for I in [BEGIN, END).
template <int I, int END, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < END) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, END>(f);
    }
}

template <int N, bool INV, typename T> struct RegDFT {
    static __device__ __forceinline__ void run(C<T>* v) {
        static_assert(N % 16 == 0 && N > 16, "composite codelet");
        constexpr int B = N / 16;
        C<T> t[B][16];
#pragma unroll
        for (int b = 0; b < B; ++b) {
#pragma unroll
            for (int a = 0; a < 16; ++a) t[b][a] = v[b + B * a];
            dft16<T, INV>(t[b]);
        }
        static_for<1, B>([&](auto bc) {
            constexpr int b = decltype(bc)::value;
            static_for<1, 16>([&](auto kc) {
                constexpr int k1 = decltype(kc)::value;
                constexpr double c = cos2pi(b * k1, N);
                constexpr double s = sin2pi(b * k1, N);
                t[b][k1] = rotw<T, INV>(t[b][k1], (T)c, (T)s);
            });
        });
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) {
            C<T> u[B];
#pragma unroll
            for (int b = 0; b < B; ++b) u[b] = t[b][k1];
            RegDFT<B, INV, T>::run(u);
#pragma unroll
            for (int k2 = 0; k2 < B; ++k2) v[k1 + 16 * k2] = u[k2];
        }
    }
};
template <bool INV, typename T> struct RegDFT<2, INV, T> {
    static __device__ __forceinline__ void run(C<T>* v) { dft2<T, INV>(v); }
};
template <bool INV, typename T> struct RegDFT<4, INV, T> {
    static __device__ __forceinline__ void run(C<T>* v) { dft4<T, INV>(v); }
};
template <bool INV, typename T> struct RegDFT<8, INV, T> {
    static __device__ __forceinline__ void run(C<T>* v) { dft8<T, INV>(v); }
};
template <bool INV, typename T> struct RegDFT<16, INV, T> {
    static __device__ __forceinline__ void run(C<T>* v) { dft16<T, INV>(v); }
};

}  // namespace se2c
