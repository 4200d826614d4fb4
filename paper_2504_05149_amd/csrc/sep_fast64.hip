// Register-resident FP64 pass kernels for separable kernel tables (the FP64 path of the
// three-pass schedule: x rows, then y and theta pencils; each pass a 1-D circular
// convolution, DFT -> product with the table's 1-D factor / L -> inverse DFT).
//
// The FP32 kernels of sep_fast.hip with complex values in double: a line of L points is
// split R1 x R2 (R1 values per thread, R2 threads per line, R1 >= R2); first-stage
// radix-R1 DFTs in registers, twiddles w_L^{t k1}, an LDS exchange, radix-R2 DFTs of the
// CC = R1 / R2 columns a thread owns (one column at a time), the product, and the
// mirror-image inverse.  Two real lines
// are packed as one complex line: rows 2s and 2s+1 (x rows) or columns 2c and 2c+1 (a
// double2 load, pencils).  One tile per workgroup.  The exchange buffer holds doubles (the
// real parts cross, then the imaginary parts), and the pencils keep one twiddle table for
// both stages: at 512 points that is 54 KB of LDS per workgroup and three workgroups per
// CU, where complex slots and two twiddle layouts (98 KB) left one (512 x 512 x 128 x 4
// FP64: y pass 715 -> 431 us, x rows 610 -> 416 us).
#include "fast_common.hpp"
#include "regfft.hpp"
#include "sep_fast64.hpp"

namespace se2c {

using D2 = double2;

__device__ __forceinline__ D2 chain_factor64(const void* const* tabs, int ntab, int i, double scale, int conj) {
    D2 v = make_double2(scale, 0.0);
    for (int j = 0; j < ntab; ++j) v = mul<double>(v, reinterpret_cast<const D2*>(tabs[j])[i]);
    if (conj) v.y = -v.y;
    return v;
}

template <int L> struct Geom64 {
    static constexpr int R1 = L > 256 ? 32 : 16;
    static constexpr int R2 = L / R1;
    static constexpr int CC = R1 / R2;
    static_assert(R1 * R2 == L && CC * R2 == R1, "line geometry");
};

// Position of element (k1, t) of one exchange line (XOR swizzle as in the FP32 kernels).
template <int R1, int R2>
__device__ __forceinline__ int xpos64(int k1, int t) {
    return k1 * R2 + (t ^ (k1 / (R1 / R2)));
}

// One line exchange: v[R1] (first stage done, in the thread's registers) -> second stage,
// product with f (the line factor, L entries), inverse second stage -> v (ready for the
// inverse first stage).  line points to the line's LDS slots (one double each, stride `ls`
// between slots): the real parts cross first, then the imaginary parts, so the exchange
// buffer holds doubles, half the LDS of complex slots.  That is what lets two or three
// workgroups share a CU at 512 points, where one workgroup with complex slots had the CU to
// itself.  While the columns are transformed the thread's R1 first-stage values are dead
// (they are in LDS and in its CC columns), so the split costs no registers.
// twf(t, k1) and twi(tt, k1) give the twiddle w_L^{t k1} (t k1 < L).
template <int L, typename TF, typename TI>
__device__ __forceinline__ void line_middle64(D2* v, double* line, int ls, const D2* f, TF twf, TI twi, int t) {
    using Gm = Geom64<L>;
    constexpr int R1 = Gm::R1, R2 = Gm::R2, CC = Gm::CC;
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1) v[k1] = mul<double>(v[k1], twf(t, k1));
    D2 u[CC][R2];
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) line[xpos64<R1, R2>(k1, t) * ls] = v[k1].x;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < CC; ++j)
#pragma unroll
        for (int tt = 0; tt < R2; ++tt) u[j][tt].x = line[xpos64<R1, R2>(CC * t + j, tt) * ls];
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) line[xpos64<R1, R2>(k1, t) * ls] = v[k1].y;
    __syncthreads();
    // each thread reads and writes back only its own CC columns; a finished column's
    // imaginary parts go straight back to its slots, so one column's values and the real
    // parts of the others are what is live
#pragma unroll
    for (int j = 0; j < CC; ++j) {
        const int k1 = CC * t + j;
#pragma unroll
        for (int tt = 0; tt < R2; ++tt) u[j][tt].y = line[xpos64<R1, R2>(k1, tt) * ls];
        RegDFT<R2, false, double>::run(u[j]);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) u[j][k2] = mul<double>(u[j][k2], f[k1 + R1 * k2]);
        RegDFT<R2, true, double>::run(u[j]);
#pragma unroll
        for (int tt = 1; tt < R2; ++tt) u[j][tt] = mulc<double>(u[j][tt], twi(tt, k1));
#pragma unroll
        for (int tt = 0; tt < R2; ++tt) line[xpos64<R1, R2>(k1, tt) * ls] = u[j][tt].y;
    }
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) v[k1].y = line[xpos64<R1, R2>(k1, t) * ls];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < CC; ++j)
#pragma unroll
        for (int tt = 0; tt < R2; ++tt) line[xpos64<R1, R2>(CC * t + j, tt) * ls] = u[j][tt].x;
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) v[k1].x = line[xpos64<R1, R2>(k1, t) * ls];
}

template <int L>
__device__ __forceinline__ void load_line_factor64(D2* f, const void* const* tabs, int ntab, int conj, int tid,
                                                   int nthr) {
    for (int i = tid; i < L; i += nthr) f[i] = chain_factor64(tabs, ntab, i, 1.0 / L, conj);
}

// x rows: one workgroup per (y-pair, G theta rows); rows 2s and 2s+1 as re/im.
template <int NX> struct RowGeom64 {
    static constexpr int G = 8;
    static constexpr int NT = G * Geom64<NX>::R2;
    static constexpr int P = NX + 1;  // LDS pitch between rows (doubles)
};

template <int NX>
__global__ void __launch_bounds__(RowGeom64<NX>::NT) x_rows_f64(Fast64Args a) {
    using Gm = Geom64<NX>;
    using RG = RowGeom64<NX>;
    constexpr int R1 = Gm::R1, R2 = Gm::R2, G = RG::G, P = RG::P;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    D2* fx = reinterpret_cast<D2*>(smem_raw);  // NX
    double* buf = reinterpret_cast<double*>(fx + NX);  // G x P
    const int tid = threadIdx.x;
    const int nslab = a.ny / 2;
    const int trows = a.m / G;
    const int per_item = nslab * trows;
    const int item = blockIdx.x / per_item;
    const int rem = blockIdx.x - item * per_item;
    const int tr = rem / nslab;
    const int s = rem - tr * nslab;
    load_line_factor64<NX>(fx, a.tab, a.ntab, a.conj_tab, tid, RG::NT);
    const int t = tid % R2, g = tid / R2;
    const int pl = NX * a.ny;
    const long long base = (long long)item * a.n + (long long)(tr * G + g) * pl + (long long)(2 * s) * NX;
    const double* in0 = a.in + base;
    const double* in1 = in0 + NX;
    D2 v[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r)
        v[r] = make_double2(__builtin_nontemporal_load(in0 + t + R2 * r), __builtin_nontemporal_load(in1 + t + R2 * r));
    __syncthreads();
    RegDFT<R1, false, double>::run(v);
    const D2* tw = a.tw;
    line_middle64<NX>(v, buf + g * P, 1, fx, [tw](int t_, int k_) { return tw[t_ * k_]; },
                      [tw](int t_, int k_) { return tw[t_ * k_]; }, t);
    RegDFT<R1, true, double>::run(v);
    double* out0 = a.out + base;
    double* out1 = out0 + NX;
#pragma unroll
    for (int r = 0; r < R1; ++r) {
        __builtin_nontemporal_store(v[r].x, out0 + t + R2 * r);
        __builtin_nontemporal_store(v[r].y, out1 + t + R2 * r);
    }
}

// Pencils: W adjacent x-pairs (double2 columns) x L points along y (axis 1) or theta
// (axis 2), in place on a.out.
template <int L> struct PencilGeom64 {
    // 16 columns (256-byte row segments) up to 128 points: 415 against 483-503 us for the
    // theta pass of 512 x 512 x 128 x 4; 8 at 256 and 512, where LDS holds the lines
    static constexpr int W = L <= 128 ? 16 : 8;
    static constexpr int NT = W * Geom64<L>::R2;
    static constexpr int P = W + 1;  // LDS pitch between line slots (doubles)
    // twiddles w_L^{t k1} in LDS as [k1][t] with pitch R2 + 1: the first stage reads
    // consecutive t at one k1, the column phase one t at the k1 = CC t + j of each thread
    // (stride CC (R2 + 1) slots), both without bank conflicts; one table for both reads
    static constexpr int TP = Geom64<L>::R2 + 1;
};

template <int L>
__global__ void __launch_bounds__(PencilGeom64<L>::NT) pencil_f64(Fast64Args a) {
    using Gm = Geom64<L>;
    using PG = PencilGeom64<L>;
    constexpr int R1 = Gm::R1, R2 = Gm::R2, W = PG::W, P = PG::P;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int TP = PG::TP;
    D2* fl = reinterpret_cast<D2*>(smem_raw);
    D2* tw2 = fl + L;                                         // [k1][t], pitch TP
    double* buf = reinterpret_cast<double*>(tw2 + R1 * TP);  // [slot][W] with pitch P
    const int tid = threadIdx.x;
    load_line_factor64<L>(fl, a.tab, a.ntab, a.conj_tab, tid, PG::NT);
    for (int i = tid; i < L; i += PG::NT) {
        const int k1 = i / R2, tt = i - k1 * R2;
        tw2[k1 * TP + tt] = a.tw[tt * k1];
    }
    const int q = tid % W, t = tid / W;
    const int ncols = a.nx / 2;
    const int ctiles = ncols / W;
    const int nouter = a.axis == 1 ? a.m : a.ny;
    const int per_item = ctiles * nouter;
    const int item = blockIdx.x / per_item;
    const int rem = blockIdx.x - item * per_item;
    const int o = rem / ctiles;
    const int ct = rem - o * ctiles;
    const int lstride = a.axis == 1 ? ncols : ncols * a.ny;            // double2 units
    const long long ostride = a.axis == 1 ? (long long)ncols * a.ny : (long long)ncols;
    D2* base = reinterpret_cast<D2*>(a.out + (long long)item * a.n) + (long long)o * ostride + ct * W + q;
    D2 v[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) v[r] = base[(long long)(t + R2 * r) * lstride];
    __syncthreads();
    RegDFT<R1, false, double>::run(v);
    const auto twl = [tw2](int t_, int k_) { return tw2[k_ * TP + t_]; };
    line_middle64<L>(v, buf + q, P, fl, twl, twl, t);
    RegDFT<R1, true, double>::run(v);
#pragma unroll
    for (int r = 0; r < R1; ++r) base[(long long)(t + R2 * r) * lstride] = v[r];
}

template <int NX>
static size_t rows64_lds() {
    return sizeof(double) * (size_t)RowGeom64<NX>::G * RowGeom64<NX>::P + sizeof(D2) * NX;
}
template <int L>
static size_t pencil64_lds() {
    using PG = PencilGeom64<L>;
    return sizeof(double) * (size_t)L * PG::P + sizeof(D2) * ((size_t)L + (size_t)Geom64<L>::R1 * PG::TP);
}

static bool len64_ok(int l) { return l == 32 || l == 64 || l == 128 || l == 256 || l == 512; }

bool fast64_supported(int nx, int ny, int m) {
    return (nx == 64 || nx == 128 || nx == 256 || nx == 512) && (nx / 2) % 16 == 0 && len64_ok(ny) &&
           len64_ok(m) && m % RowGeom64<64>::G == 0;
}

template <int NX>
static hipError_t rows64_t(const Fast64Args& a, hipStream_t s) {
    const int nblocks = (a.ny / 2) * (a.m / RowGeom64<NX>::G) * a.nitems;
    hipLaunchKernelGGL((x_rows_f64<NX>), dim3(nblocks), dim3(RowGeom64<NX>::NT), rows64_lds<NX>(), s, a);
    return hipGetLastError();
}

template <int L>
static hipError_t pencil64_t(const Fast64Args& a, hipStream_t s) {
    const int nouter = a.axis == 1 ? a.m : a.ny;
    const int nblocks = ((a.nx / 2) / PencilGeom64<L>::W) * nouter * a.nitems;
    hipLaunchKernelGGL((pencil_f64<L>), dim3(nblocks), dim3(PencilGeom64<L>::NT), pencil64_lds<L>(), s, a);
    return hipGetLastError();
}

hipError_t launch_rows_f64(const Fast64Args& a, hipStream_t s) {
    switch (a.nx) {
        case 64: return rows64_t<64>(a, s);
        case 128: return rows64_t<128>(a, s);
        case 256: return rows64_t<256>(a, s);
        case 512: return rows64_t<512>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_pencil_f64(const Fast64Args& a, hipStream_t s) {
    switch (a.axis == 1 ? a.ny : a.m) {
        case 32: return pencil64_t<32>(a, s);
        case 64: return pencil64_t<64>(a, s);
        case 128: return pencil64_t<128>(a, s);
        case 256: return pencil64_t<256>(a, s);
        case 512: return pencil64_t<512>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t prepare_fast64_kernels() {
    hipError_t e = hipSuccess;
#define SE2C_A64(K, B)                                                                                           \
    if (e == hipSuccess)                                                                                         \
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(K), hipFuncAttributeMaxDynamicSharedMemorySize, (int)(B));
    SE2C_A64(x_rows_f64<64>, rows64_lds<64>()) SE2C_A64(x_rows_f64<128>, rows64_lds<128>())
    SE2C_A64(x_rows_f64<256>, rows64_lds<256>()) SE2C_A64(x_rows_f64<512>, rows64_lds<512>())
    SE2C_A64(pencil_f64<32>, pencil64_lds<32>()) SE2C_A64(pencil_f64<64>, pencil64_lds<64>())
    SE2C_A64(pencil_f64<128>, pencil64_lds<128>()) SE2C_A64(pencil_f64<256>, pencil64_lds<256>())
    SE2C_A64(pencil_f64<512>, pencil64_lds<512>())
#undef SE2C_A64
    return e;
}

}  // namespace se2c
