// In-register DFT codelets with compile-time twiddles (FP32/FP64).
//
// RegDFT<N, INV>(v): natural-order in, natural-order out, v[0..N-1] held in
// registers (every index is a compile-time constant after unrolling).  N = 2, 3, 4, 5,
// 7, 8, 16 use the hand-written butterflies of fft_device.hpp; composite N = A * B
// (A = 16, 8, 4 or 2, or for odd N 3, 5 or 7; B = N / A, e.g. 32 = 16 x 2, 96 = 16 x 6,
// 6 = 2 x 3, 15 = 3 x 5) is composed
// as B A-point DFTs on the stride-B subsequences, twiddles w_N^{b k1}, then A B-point
// DFTs.  The codelet twiddles are evaluated at compile
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

// Composite size N = A * B: A-point DFTs on the B stride-B subsequences, twiddles
// w_N^{b k1}, then A B-point DFTs (decimation in time).  A is 16 when 16 divides N,
// else the largest of 8, 4, 2 dividing N; sizes 3 * 2^k end in the radix-3 codelet.
template <int N> struct RegSplit {
    static constexpr int A = (N % 16 == 0) ? 16
                             : (N % 8 == 0) ? 8
                             : (N % 4 == 0) ? 4
                             : (N % 2 == 0) ? 2
                             : (N % 3 == 0) ? 3   // odd composites: 9 = 3 x 3, 15 = 3 x 5, 21 = 3 x 7
                             : (N % 5 == 0) ? 5
                                            : 7;
    static constexpr int B = N / A;
};

template <int N, bool INV, typename T> struct RegDFT {
    static __device__ __forceinline__ void run(C<T>* v) {
        constexpr int A = RegSplit<N>::A;
        constexpr int B = RegSplit<N>::B;
        static_assert(A * B == N && B > 1, "composite codelet");
        C<T> t[B][A];
#pragma unroll
        for (int b = 0; b < B; ++b) {
#pragma unroll
            for (int a = 0; a < A; ++a) t[b][a] = v[b + B * a];
            RegDFT<A, INV, T>::run(t[b]);
        }
        static_for<1, B>([&](auto bc) {
            constexpr int b = decltype(bc)::value;
            static_for<1, A>([&](auto kc) {
                constexpr int k1 = decltype(kc)::value;
                constexpr double c = cos2pi(b * k1, N);
                constexpr double s = sin2pi(b * k1, N);
                t[b][k1] = rotw<T, INV>(t[b][k1], (T)c, (T)s);
            });
        });
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
            C<T> u[B];
#pragma unroll
            for (int b = 0; b < B; ++b) u[b] = t[b][k1];
            RegDFT<B, INV, T>::run(u);
#pragma unroll
            for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = u[k2];
        }
    }
};
template <bool INV, typename T> struct RegDFT<3, INV, T> {
    static __device__ __forceinline__ void run(C<T>* v) { dft3<T, INV>(v); }
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
template <bool INV, typename T> struct RegDFT<5, INV, T> {
    static __device__ __forceinline__ void run(C<T>* v) { dft5<T, INV>(v); }
};
template <bool INV, typename T> struct RegDFT<7, INV, T> {
    static __device__ __forceinline__ void run(C<T>* v) { dft7<T, INV>(v); }
};

}  // namespace se2c
