// Device-side FFT building blocks for gfx950 (CDNA4, wave64).
//
// Stockham auto-sort radix-R stages over an LDS-resident tile of complex lines.
// A stage reads R points per butterfly at stride L/R, applies the twiddles
// w_L^{r*k*L/(Ns*R)} (k = j mod Ns, Ns = product of earlier radices), does an
// in-register radix-R DFT and writes the R results at stride Ns; after the last
// stage the line is in natural frequency order.  Every thread first reads all of
// its butterflies into registers, the workgroup synchronises, then writes, so a
// single LDS buffer serves as both source and destination.
//
// The forward transform uses e^{-2 pi i jk/L} as in the paper's DFT (Sec. 2.3,
// eq. (3DFT)); the inverse uses the conjugate roots and no 1/L (the scale is
// folded into the spectral product).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace se2c {

template <typename T> struct cx;
template <> struct cx<float> { using t = float2; };
template <> struct cx<double> { using t = double2; };
template <typename T> using C = typename cx<T>::t;

template <typename T> __device__ __forceinline__ C<T> mk(T a, T b) { C<T> r; r.x = a; r.y = b; return r; }
template <typename T> __device__ __forceinline__ C<T> add(C<T> a, C<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ C<T> sub(C<T> a, C<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ C<T> mul(C<T> a, C<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T> __device__ __forceinline__ C<T> mulc(C<T> a, C<T> b) {
    return mk<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T> __device__ __forceinline__ C<T> scl(C<T> a, T s) { return mk<T>(a.x * s, a.y * s); }

// Multiply by -i (forward) or +i (inverse).
template <typename T, bool INV> __device__ __forceinline__ C<T> rot(C<T> a) {
    return INV ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}
// Multiply by w = (c, -s) forward or (c, +s) inverse, i.e. e^{-+i phi} with c=cos, s=sin.
template <typename T, bool INV> __device__ __forceinline__ C<T> rotw(C<T> a, T c, T s) {
    return INV ? mk<T>(a.x * c - a.y * s, a.x * s + a.y * c)
               : mk<T>(a.x * c + a.y * s, a.y * c - a.x * s);
}

// Constants written in double and rounded to T.
#define SE2C_SQRT1_2 0.70710678118654752440084436210484903928
#define SE2C_COS_PI8 0.92387953251128675612818318939678828682
#define SE2C_SIN_PI8 0.38268343236508977172845998403039886676
#define SE2C_SQRT3_2 0.86602540378443864676372317075293618347
// cos and sin of 2 pi j / 5 and 2 pi j / 7
#define SE2C_C5_1 0.30901699437494742410229341718281905886
#define SE2C_C5_2 -0.80901699437494742410229341718281905886
#define SE2C_S5_1 0.95105651629515357211643933337938214340
#define SE2C_S5_2 0.58778525229247312916870595463907276860
#define SE2C_C7_1 0.62348980185873353052500488400423981063
#define SE2C_C7_2 -0.22252093395631440428890256449679475947
#define SE2C_C7_3 -0.90096886790241912623610231950744505117
#define SE2C_S7_1 0.78183148246802980870844452667405775023
#define SE2C_S7_2 0.97492791218182360701813168299393121723
#define SE2C_S7_3 0.43388373911755812047576833284835875461

template <typename T, bool INV> __device__ __forceinline__ void dft2(C<T>* a) {
    C<T> t = a[0];
    a[0] = add<T>(t, a[1]);
    a[1] = sub<T>(t, a[1]);
}

template <typename T, bool INV> __device__ __forceinline__ void dft3(C<T>* a) {
    const T h = (T)SE2C_SQRT3_2;
    C<T> s = add<T>(a[1], a[2]);
    C<T> d = sub<T>(a[1], a[2]);
    C<T> m = mk<T>(a[0].x - (T)0.5 * s.x, a[0].y - (T)0.5 * s.y);
    // -i*h*d (forward) / +i*h*d (inverse)
    C<T> r = rot<T, INV>(scl<T>(d, h));
    a[0] = add<T>(a[0], s);
    a[1] = add<T>(m, r);
    a[2] = sub<T>(m, r);
}

// Odd prime length P: X_k = b_k + (-+i) d_k and X_{P-k} = b_k - (-+i) d_k with
// b_k = a_0 + sum_j cos(2 pi jk/P) (a_j + a_{P-j}), d_k = sum_j sin(2 pi jk/P) (a_j - a_{P-j}).
template <typename T, bool INV> __device__ __forceinline__ void dft5(C<T>* a) {
    const T c1 = (T)SE2C_C5_1, c2 = (T)SE2C_C5_2, s1 = (T)SE2C_S5_1, s2 = (T)SE2C_S5_2;
    const C<T> p1 = add<T>(a[1], a[4]), m1 = sub<T>(a[1], a[4]);
    const C<T> p2 = add<T>(a[2], a[3]), m2 = sub<T>(a[2], a[3]);
    const C<T> b1 = mk<T>(a[0].x + c1 * p1.x + c2 * p2.x, a[0].y + c1 * p1.y + c2 * p2.y);
    const C<T> b2 = mk<T>(a[0].x + c2 * p1.x + c1 * p2.x, a[0].y + c2 * p1.y + c1 * p2.y);
    const C<T> d1 = rot<T, INV>(mk<T>(s1 * m1.x + s2 * m2.x, s1 * m1.y + s2 * m2.y));
    const C<T> d2 = rot<T, INV>(mk<T>(s2 * m1.x - s1 * m2.x, s2 * m1.y - s1 * m2.y));
    a[0] = add<T>(a[0], add<T>(p1, p2));
    a[1] = add<T>(b1, d1);
    a[4] = sub<T>(b1, d1);
    a[2] = add<T>(b2, d2);
    a[3] = sub<T>(b2, d2);
}

template <typename T, bool INV> __device__ __forceinline__ void dft7(C<T>* a) {
    const T c1 = (T)SE2C_C7_1, c2 = (T)SE2C_C7_2, c3 = (T)SE2C_C7_3;
    const T s1 = (T)SE2C_S7_1, s2 = (T)SE2C_S7_2, s3 = (T)SE2C_S7_3;
    const C<T> p1 = add<T>(a[1], a[6]), m1 = sub<T>(a[1], a[6]);
    const C<T> p2 = add<T>(a[2], a[5]), m2 = sub<T>(a[2], a[5]);
    const C<T> p3 = add<T>(a[3], a[4]), m3 = sub<T>(a[3], a[4]);
    // cos(2 pi jk/7) and sin(2 pi jk/7) for k = 1, 2, 3 (jk reduced mod 7; sin is odd)
    const C<T> b1 = mk<T>(a[0].x + c1 * p1.x + c2 * p2.x + c3 * p3.x, a[0].y + c1 * p1.y + c2 * p2.y + c3 * p3.y);
    const C<T> b2 = mk<T>(a[0].x + c2 * p1.x + c3 * p2.x + c1 * p3.x, a[0].y + c2 * p1.y + c3 * p2.y + c1 * p3.y);
    const C<T> b3 = mk<T>(a[0].x + c3 * p1.x + c1 * p2.x + c2 * p3.x, a[0].y + c3 * p1.y + c1 * p2.y + c2 * p3.y);
    const C<T> d1 = rot<T, INV>(mk<T>(s1 * m1.x + s2 * m2.x + s3 * m3.x, s1 * m1.y + s2 * m2.y + s3 * m3.y));
    const C<T> d2 = rot<T, INV>(mk<T>(s2 * m1.x - s3 * m2.x - s1 * m3.x, s2 * m1.y - s3 * m2.y - s1 * m3.y));
    const C<T> d3 = rot<T, INV>(mk<T>(s3 * m1.x - s1 * m2.x + s2 * m3.x, s3 * m1.y - s1 * m2.y + s2 * m3.y));
    a[0] = add<T>(a[0], add<T>(p1, add<T>(p2, p3)));
    a[1] = add<T>(b1, d1);
    a[6] = sub<T>(b1, d1);
    a[2] = add<T>(b2, d2);
    a[5] = sub<T>(b2, d2);
    a[3] = add<T>(b3, d3);
    a[4] = sub<T>(b3, d3);
}

template <typename T, bool INV> __device__ __forceinline__ void dft4(C<T>* a) {
    C<T> t0 = add<T>(a[0], a[2]);
    C<T> t1 = sub<T>(a[0], a[2]);
    C<T> t2 = add<T>(a[1], a[3]);
    C<T> t3 = rot<T, INV>(sub<T>(a[1], a[3]));
    a[0] = add<T>(t0, t2);
    a[2] = sub<T>(t0, t2);
    a[1] = add<T>(t1, t3);
    a[3] = sub<T>(t1, t3);
}

template <typename T, bool INV> __device__ __forceinline__ void dft8(C<T>* a) {
    C<T> e[4] = {a[0], a[2], a[4], a[6]};
    C<T> o[4] = {a[1], a[3], a[5], a[7]};
    dft4<T, INV>(e);
    dft4<T, INV>(o);
    const T r = (T)SE2C_SQRT1_2;
    o[1] = rotw<T, INV>(o[1], r, r);        // w8^1
    o[2] = rot<T, INV>(o[2]);               // w8^2 = -i
    o[3] = rotw<T, INV>(o[3], -r, r);       // w8^3
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        a[k] = add<T>(e[k], o[k]);
        a[k + 4] = sub<T>(e[k], o[k]);
    }
}

template <typename T, bool INV> __device__ __forceinline__ void dft16(C<T>* a) {
    // 16 = 4 x 4: column DFTs over n1, twiddle w16^{n2 k1}, row DFTs over n2.
    C<T> y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        C<T> t[4] = {a[n2], a[4 + n2], a[8 + n2], a[12 + n2]};
        dft4<T, INV>(t);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = t[k1];
    }
    const T c1 = (T)SE2C_COS_PI8, s1 = (T)SE2C_SIN_PI8, r = (T)SE2C_SQRT1_2;
    // n2 = 1: w^1, w^2, w^3 ; n2 = 2: w^2, w^4, w^6 ; n2 = 3: w^3, w^6, w^9
    y[1][1] = rotw<T, INV>(y[1][1], c1, s1);
    y[1][2] = rotw<T, INV>(y[1][2], r, r);
    y[1][3] = rotw<T, INV>(y[1][3], s1, c1);
    y[2][1] = rotw<T, INV>(y[2][1], r, r);
    y[2][2] = rot<T, INV>(y[2][2]);
    y[2][3] = rotw<T, INV>(y[2][3], -r, r);
    y[3][1] = rotw<T, INV>(y[3][1], s1, c1);
    y[3][2] = rotw<T, INV>(y[3][2], -r, r);
    y[3][3] = rotw<T, INV>(y[3][3], -c1, -s1);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        C<T> t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
        dft4<T, INV>(t);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = t[k2];
    }
}

template <int R, typename T, bool INV> __device__ __forceinline__ void dftR(C<T>* a) {
    if constexpr (R == 2) dft2<T, INV>(a);
    else if constexpr (R == 3) dft3<T, INV>(a);
    else if constexpr (R == 4) dft4<T, INV>(a);
    else if constexpr (R == 5) dft5<T, INV>(a);
    else if constexpr (R == 7) dft7<T, INV>(a);
    else if constexpr (R == 8) dft8<T, INV>(a);
    else dft16<T, INV>(a);
}

// Signed frequency of DFT index t on a length-L axis: t for t <= (L-1)/2, else t - L.
// For odd L = 2K+1 this is the set |k| <= K; for even L it is {-L/2, ..., L/2-1}, and
// (-1)^k of the signed frequency equals (-1)^t only when L is even.
__host__ __device__ inline int signed_freq(int t, int L) { return t <= (L - 1) / 2 ? t : t - L; }

// Zero padding from a length-L spectrum to a length-G one (G >= L): the L-index that G-index
// g takes its value from (-1: none, the value is zero), keeping every signed frequency
// |k| <= (L-1)/2 (odd L).  For even L the index L/2 holds +-L/2 together; when G > L it is
// split in halves between tau_G(-L/2) and tau_G(+L/2) (*half set), when G = L kept whole.
__device__ __forceinline__ int pad_source(int g, int G, int L, bool* half) {
    const int k = signed_freq(g, G);
    *half = false;
    if (L & 1) {
        const int K = (L - 1) / 2;
        if (k < -K || k > K) return -1;
        return k < 0 ? k + L : k;
    }
    const int h = L / 2;
    if (k > -h && k < h) return k < 0 ? k + L : k;
    if (k == h || k == -h) {
        *half = G > L;
        return h;
    }
    return -1;
}

// Division by a runtime divisor 1 <= d < 2^16 of n < 2^16 (every index of a tile:
// tiles hold at most 16384 points): q = mulhi(n, m) with m = ceil(2^32 / d).  With
// m d = 2^32 + r, 0 <= r < d, n m / 2^32 = n/d + n r / (d 2^32) and the second term
// is below 2^-16 < 1/d, so the floor is exact.  d = 1 is m = 0.  Building m takes one
// 32-bit division (a 64-bit magic number would take a software 64-bit division on
// the scalar unit per stage).
struct FastDiv {
    uint32_t m;
};
__host__ __device__ inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    f.m = d > 1 ? 0xFFFFFFFFu / d + 1u : 0u;
    return f;
}
__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) {
    return f.m ? __umulhi(n, f.m) : n;
}

// One radix-R stage over 'nlines' lines of length L in LDS.
// Element (line, e) lives at buf[line*ls + e*es].  'line_fast' selects whether
// consecutive threads walk consecutive lines (use when ls == 1) or consecutive
// butterflies within a line (use when es == 1).
struct StageGeom {
    int L, Ns, es, ls, nlines;
    FastDiv div_nbl;  // L/R (butterflies per line)
    FastDiv div_ns;   // Ns
    FastDiv div_nl;   // nlines
    FastDiv div_l;    // L
    int tw_step;      // L/(Ns*R)
};

template <typename T, int R, int MAXV, bool INV>
__device__ __forceinline__ void stockham_stage(C<T>* buf, const C<T>* tw, const StageGeom g,
                                               bool line_fast, int tid, int nthr) {
    constexpr int U = (MAXV + R - 1) / R;
    const int nbl = g.L / R;
    const int nb = nbl * g.nlines;
    C<T> v[U][R];
    int dst[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int b = tid + u * nthr;
        dst[u] = -1;
        if (b < nb) {
            int line, j;
            if (line_fast) {
                j = (int)fdiv((uint32_t)b, g.div_nl);
                line = b - j * g.nlines;
            } else {
                line = (int)fdiv((uint32_t)b, g.div_nbl);
                j = b - line * nbl;
            }
            const int jq = (int)fdiv((uint32_t)j, g.div_ns);
            const int k = j - jq * g.Ns;
            const C<T>* src = buf + line * g.ls + j * g.es;
#pragma unroll
            for (int r = 0; r < R; ++r) v[u][r] = src[r * nbl * g.es];
            if (g.Ns > 1) {
                const int step = k * g.tw_step;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C<T> w = tw[r * step];
                    v[u][r] = INV ? mulc<T>(v[u][r], w) : mul<T>(v[u][r], w);
                }
            }
            dftR<R, T, INV>(v[u]);
            dst[u] = line * g.ls + (jq * g.Ns * R + k) * g.es;
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (dst[u] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[dst[u] + r * g.Ns * g.es] = v[u][r];
        }
    }
    __syncthreads();
}

// One radix-R stage by direct summation, for prime R without a codelet.  Output
// rr of butterfly j (k = j mod Ns) is sum_r v_r w_L^{r k L/(Ns R)} w_R^{r rr}
// = sum_r v_r w_L^{r (k L/(Ns R) + rr L/R) mod L}: one table twiddle per term, O(R)
// work per point.  Every thread computes up to MAXV outputs (the tile holds at
// most MAXV points per thread), the workgroup synchronises, then they are written.
template <typename T, int MAXV, bool INV>
__device__ __forceinline__ void direct_stage(C<T>* buf, const C<T>* tw, const StageGeom g, int R, bool line_fast,
                                             int tid, int nthr) {
    const int nbl = g.L / R;
    const int total = g.L * g.nlines;
    // element e -> (line, output rr, butterfly j = jq Ns + k)
    auto split = [&](int e, int& line, int& rr, int& j, int& jq, int& k) {
        int q;
        if (line_fast) {
            q = (int)fdiv((uint32_t)e, g.div_nl);
            line = e - q * g.nlines;
        } else {
            line = (int)fdiv((uint32_t)e, g.div_l);
            q = e - line * g.L;
        }
        rr = (int)fdiv((uint32_t)q, g.div_nbl);
        j = q - rr * nbl;
        jq = (int)fdiv((uint32_t)j, g.div_ns);
        k = j - jq * g.Ns;
    };
    C<T> acc[MAXV];
#pragma unroll
    for (int u = 0; u < MAXV; ++u) {
        const int e = tid + u * nthr;
        acc[u] = mk<T>((T)0, (T)0);
        if (e < total) {
            int line, rr, j, jq, k;
            split(e, line, rr, j, jq, k);
            const C<T>* src = buf + line * g.ls + j * g.es;
            const int step = k * g.tw_step + rr * nbl;  // < L
            int idx = 0;
            C<T> sum = mk<T>((T)0, (T)0);
            for (int r = 0; r < R; ++r) {
                const C<T> v = src[r * nbl * g.es];
                const C<T> w = tw[idx];
                sum = add<T>(sum, INV ? mulc<T>(v, w) : mul<T>(v, w));
                idx += step;
                if (idx >= g.L) idx -= g.L;
            }
            acc[u] = sum;
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MAXV; ++u) {
        const int e = tid + u * nthr;
        if (e < total) {
            int line, rr, j, jq, k;
            split(e, line, rr, j, jq, k);
            buf[line * g.ls + (jq * g.Ns * R + k + rr * g.Ns) * g.es] = acc[u];
        }
    }
    __syncthreads();
}

// Radix plan for one transform length: up to 8 stages.  For a prime length L above
// 7 (rader = 1) the stages are those of L - 1: the DFT runs as Rader's cyclic
// convolution of length L - 1, with its tables at rtab (device, the kernel's type):
// the twiddles w_{L-1}^j, the forward and inverse kernel spectra (each L - 1 complex
// values), then the index maps g^q mod L and g^-q mod L (L - 1 ints each).
struct RadixPlan {
    int L;
    int nst;
    int r[8];
    int rader;
    const void* rtab;
};

// Entries of the twiddle table a plan's stages read: L, or L - 1 under Rader.
__host__ __device__ __forceinline__ int stage_tw_len(const RadixPlan& p) { return p.rader ? p.L - 1 : p.L; }

// Complex slots of the LDS copy of a plan's tables, for complex values of cb bytes:
// the twiddles, and under Rader the whole table block (3 (L - 1) complex values and
// 2 (L - 1) ints), rounded up to whole slots.
__host__ __device__ __forceinline__ int tables_slots(const RadixPlan& p, int cb) {
    if (!p.rader) return p.L;
    const int n = p.L - 1;
    return 3 * n + (8 * n + cb - 1) / cb;
}

// The Stockham stages r[0..nst) of a length-L transform over 'nlines' lines in LDS.
template <typename T, int MAXV, bool INV, bool ODD>
__device__ __forceinline__ void run_stages(C<T>* buf, const C<T>* tw, const RadixPlan& p, int L, int es, int ls,
                                           int nlines, bool line_fast, int tid, int nthr) {
    int Ns = 1;
    for (int s = 0; s < p.nst; ++s) {
        const int R = p.r[s];
        StageGeom g;
        g.L = L;
        g.Ns = Ns;
        g.es = es;
        g.ls = ls;
        g.nlines = nlines;
        g.div_nbl = make_fastdiv((uint32_t)(L / R));
        g.div_ns = make_fastdiv((uint32_t)Ns);
        g.div_nl = make_fastdiv((uint32_t)nlines);
        g.div_l = make_fastdiv((uint32_t)L);
        g.tw_step = L / (Ns * R);
        switch (R) {
            case 16: stockham_stage<T, 16, MAXV, INV>(buf, tw, g, line_fast, tid, nthr); break;
            case 8: stockham_stage<T, 8, MAXV, INV>(buf, tw, g, line_fast, tid, nthr); break;
            case 4: stockham_stage<T, 4, MAXV, INV>(buf, tw, g, line_fast, tid, nthr); break;
            case 3: stockham_stage<T, 3, MAXV, INV>(buf, tw, g, line_fast, tid, nthr); break;
            case 2: stockham_stage<T, 2, MAXV, INV>(buf, tw, g, line_fast, tid, nthr); break;
            default:
                // radices other than 2^a 3^b exist only in kernels instantiated with ODD
                if constexpr (ODD) {
                    if (R == 5) stockham_stage<T, 5, MAXV, INV>(buf, tw, g, line_fast, tid, nthr);
                    else if (R == 7) stockham_stage<T, 7, MAXV, INV>(buf, tw, g, line_fast, tid, nthr);
                    else direct_stage<T, MAXV, INV>(buf, tw, g, R, line_fast, tid, nthr);
                }
                break;
        }
        Ns *= R;
    }
}

// Work item e of the n * nlines items of a line-wise step -> (line, q < n).
__device__ __forceinline__ void split_item(int e, int n, int nlines, FastDiv div_n, FastDiv div_nl, bool line_fast,
                                           int& line, int& q) {
    if (line_fast) {
        q = (int)fdiv((uint32_t)e, div_nl);
        line = e - q * nlines;
    } else {
        line = (int)fdiv((uint32_t)e, div_n);
        q = e - line * n;
    }
}

template <typename T>
__device__ __forceinline__ C<T> conj_if(C<T> v, bool c) {
    if (c) v.y = -v.y;
    return v;
}

// Rader's reindexing of a prime-length line: GATHER moves x[g^q] to slot 1 + q (and
// conjugates it when CONJ), otherwise slot 1 + q (conjugated when CONJ) moves to
// g^-q.  Slot 0 stays.  Every value passes through registers between two barriers,
// so the permutation is in place.
template <typename T, int MAXV, bool GATHER, bool CONJ>
__device__ __forceinline__ void rader_permute(C<T>* buf, const int* perm, int n, int es, int ls, int nlines,
                                              FastDiv div_n, FastDiv div_nl, bool line_fast, int tid, int nthr) {
    const int total = n * nlines;
    C<T> v[MAXV];
#pragma unroll
    for (int u = 0; u < MAXV; ++u) {
        const int e = tid + u * nthr;
        if (e < total) {
            int line, q;
            split_item(e, n, nlines, div_n, div_nl, line_fast, line, q);
            const int src = GATHER ? perm[q] : 1 + q;
            v[u] = conj_if<T>(buf[line * ls + src * es], CONJ);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MAXV; ++u) {
        const int e = tid + u * nthr;
        if (e < total) {
            int line, q;
            split_item(e, n, nlines, div_n, div_nl, line_fast, line, q);
            const int dst = GATHER ? 1 + q : perm[q];
            buf[line * ls + dst * es] = v[u];
        }
    }
    __syncthreads();
}

// Transform 'nlines' lines of length p.L (forward or inverse) in LDS.  'tw' is the
// LDS copy of the plan's tables (tables_slots): the stage twiddles, and under Rader
// the rest of its table block after them.
//
// A prime length above 7 (ODD kernels) runs by Rader's algorithm.  With a generator
// g of the units mod L, X[g^-m] = x[0] + sum_q x[g^q] w^{g^(q-m)}: a cyclic
// convolution of length n = L - 1 of a_q = x[g^q] with b_j = w^{g^-j} (w = w_L,
// conjugated for the inverse transform).  It is computed as A = DFT_n(a), the product
// with B = DFT_n(b) / n (tabulated in FP64), and an unnormalised inverse DFT_n; x[0]
// enters as a constant added to the zero frequency of the product, and
// X[0] = x[0] + A[0].  Both length-n transforms run through the one stage loop of
// this direction: the opposite direction is its conjugate, conj(DFT(conj(v))), and
// those conjugations ride on the permutations and the product step.
template <typename T, int MAXV, bool INV, bool ODD = false>
__device__ __forceinline__ void line_fft(C<T>* buf, const C<T>* tw, const RadixPlan& p, int es, int ls, int nlines,
                                         bool line_fast, int tid, int nthr) {
    bool rad = false;
    if constexpr (ODD) rad = p.rader != 0;
    const int n = rad ? p.L - 1 : p.L;
    C<T>* sub = rad ? buf + es : buf;
    const C<T>* bh = nullptr;
    const int* pin = nullptr;
    FastDiv div_n{}, div_nl{};
    if constexpr (ODD) {
        if (rad) {
            const C<T>* tab = tw;
            bh = tab + (INV ? 2 : 1) * n;
            pin = reinterpret_cast<const int*>(tab + 3 * n);
            div_n = make_fastdiv((uint32_t)n);
            div_nl = make_fastdiv((uint32_t)nlines);
            // the forward DFT_n of an inverse transform runs as conj(DFT_n^-1(conj a))
            rader_permute<T, MAXV, true, INV>(buf, pin, n, es, ls, nlines, div_n, div_nl, line_fast, tid, nthr);
        }
    }
    const int npass = rad ? 2 : 1;
#pragma unroll 1
    for (int pass = 0; pass < npass; ++pass) {
        run_stages<T, MAXV, INV, ODD>(sub, tw, p, n, es, ls, nlines, line_fast, tid, nthr);
        if constexpr (ODD) {
            if (rad && pass == 0) {
                const int total = n * nlines;
                for (int e = tid; e < total; e += nthr) {
                    int line, k;
                    split_item(e, n, nlines, div_n, div_nl, line_fast, line, k);
                    C<T>* row = buf + line * ls;
                    const C<T> a = conj_if<T>(row[(1 + k) * es], INV);  // A[k]
                    C<T> v = mul<T>(a, bh[k]);
                    if (k == 0) {  // the only work item that touches slot 0 of this line
                        const C<T> x0 = row[0];
                        row[0] = add<T>(x0, a);
                        v = add<T>(v, x0);
                    }
                    // the inverse DFT_n of a forward transform runs as conj(DFT_n(conj v))
                    row[(1 + k) * es] = conj_if<T>(v, !INV);
                }
                __syncthreads();
            }
        }
    }
    if constexpr (ODD) {
        if (rad)
            rader_permute<T, MAXV, false, !INV>(buf, pin + n, n, es, ls, nlines, div_n, div_nl, line_fast, tid,
                                                nthr);
    }
}

// Offset of the coefficient at array indices (k3, k2, k1) in a quarter table
// [m][ny/2+1][nx/2+1]: the entry at the nonnegative signed frequencies |k1|, |k2|
// (k -> min(k, L - k); the Nyquist index of an even length maps to itself).
__device__ __forceinline__ long long quarter_offset(int kt, int ky, int kx, int nx, int ny) {
    const int ax = min(kx, nx - kx), ay = min(ky, ny - ky);
    return ((long long)kt * (ny / 2 + 1) + ay) * (nx / 2 + 1) + ax;
}

// Workgroups are handed to the chip's 8 XCDs in turn (workgroup b to XCD b mod 8), each
// XCD with its own L2.  xcd_contiguous(b, G) renumbers the G workgroups of a launch so
// that every XCD receives one contiguous range of the new indices, in its own dispatch
// order: workgroups with neighbouring indices (tiles that share table entries, or halves
// of the same cache lines) run on one XCD close together in time, and what they share is
// fetched from HBM once.  A bijection of [0, G) for every G >= 1; a grid-stride loop over
// G tiles keeps the property when its grid is a multiple of 8.
__device__ __forceinline__ int xcd_contiguous(int b, int G) {
    const int x = b & 7, i = b >> 3;
    const int per = G >> 3, rem = G & 7;
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + i;
}

}  // namespace se2c
