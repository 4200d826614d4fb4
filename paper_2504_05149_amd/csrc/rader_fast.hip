// Register-resident pencils (FP32 and FP64) for a prime line length P (the paper's odd
// grids L = 2K+1 with L prime), by Rader's algorithm.
//
// With a generator g of the units mod P and N = P - 1:
//   X[0]       = sum_n x[n],
//   X[g^-m]    = x[0] + sum_q x[g^q] w_P^{g^(q-m)}     (m = 0 .. N-1),
// a cyclic convolution of a_q = x[g^q] with b_j = w_P^{g^-j}; and for the inverse DFT of
// a spectrum given in that permuted order, Y'[m] = Y[g^-m],
//   y[0]       = Y[0] + sum_m Y'[m],
//   y[g^p]     = Y[0] + sum_m Y'[m] c_{p-m},   c_j = conj(w_P^{g^j}),
// whose DFT is conj(DFT(b)): one table B = DFT_N(b) / N (from the plan's Rader block)
// serves both.  Each length-N cyclic convolution runs as DFT_N, product, inverse DFT_N in
// registers (N = R1 x R2, R1 values per thread, R2 threads per line, one LDS exchange
// each way); the constant x[0] (or Y[0]) enters at frequency 0 of the product, which adds
// it to every output.  The y pass (forward, product with the chain, inverse) keeps the
// permuted order between its two transforms: no scatter or gather in between.
//
// MODE 0: forward DFT, product with the chain (x scale, conjugated for the adjoint),
//         inverse DFT; MODE 1: forward only; MODE 2: inverse only.  The product of MODE 0
// is the 3-D chain factor at the line's frequencies (PencilArgs mul 2: FULL, quarter or
// separable tables) or a 1-D factor along the line (mul 1: one axis of separable tables,
// a 1-D circular convolution).  Pencils on the planes of field pairs (PencilArgs mode 1):
// W columns of x at one outer coordinate, lines along y (axis 1) or theta (axis 2); or
// (axis 0, ROWS) W rows of x at one theta, lines along x.  Tiles are loaded into LDS whole, computed in registers,
// scattered back to natural order through LDS and stored.
#include "passes.hpp"
#include "regfft.hpp"

namespace se2c {

template <int P> struct RaderGeom {
    static constexpr int R1 = 0, R2 = 0;
};
// P - 1 = R1 x R2 with R2 dividing R1 (the exchange) and R1, R2 register codelets; the
// primes whose P - 1 has no such split (31, 43, 53, ...) stay on the generic kernels
template <> struct RaderGeom<13> { static constexpr int R1 = 6, R2 = 2; };
template <> struct RaderGeom<17> { static constexpr int R1 = 8, R2 = 2; };
template <> struct RaderGeom<19> { static constexpr int R1 = 6, R2 = 3; };
template <> struct RaderGeom<29> { static constexpr int R1 = 14, R2 = 2; };
template <> struct RaderGeom<37> { static constexpr int R1 = 12, R2 = 3; };
template <> struct RaderGeom<41> { static constexpr int R1 = 20, R2 = 2; };
template <> struct RaderGeom<61> { static constexpr int R1 = 30, R2 = 2; };
template <> struct RaderGeom<73> { static constexpr int R1 = 24, R2 = 3; };
template <> struct RaderGeom<97> { static constexpr int R1 = 24, R2 = 4; };
template <> struct RaderGeom<101> { static constexpr int R1 = 10, R2 = 10; };
template <> struct RaderGeom<109> { static constexpr int R1 = 36, R2 = 3; };
template <> struct RaderGeom<113> { static constexpr int R1 = 28, R2 = 4; };

constexpr int kRaderW = 32;  // columns per tile: 128-byte rows of each plane

template <typename T, int P, bool ROWS>
static constexpr size_t rader_lds() {
    constexpr int N = P - 1;
    return sizeof(C<T>) * ((size_t)P * (kRaderW + (ROWS ? 1 : 0)) + 3 * N + P) + sizeof(int) * 2 * N;
}

// The chain's factor at (kx, ky, kt) (FULL, quarter or separable tables), x scale,
// conjugated for the adjoint.
template <typename T>
__device__ __forceinline__ C<T> rader_chain_factor(const PencilArgs& a, int kx, int ky, int kt) {
    C<T> w = mk<T>((T)a.scale, (T)0);
    for (int j = 0; j < a.ntab; ++j) {
        if (a.tab3[j]) {
            const bool qj = (a.tab3_quarter >> j) & 1u;
            const int ax = qj ? min(kx, a.nx - kx) : kx;
            const int ay = qj ? min(ky, a.ny - ky) : ky;
            const long long off = ((long long)kt * (qj ? a.ny / 2 + 1 : a.ny) + ay) * (qj ? a.nx / 2 + 1 : a.nx) + ax;
            w = mul<T>(w, reinterpret_cast<const C<T>*>(a.tab3[j])[off]);
        } else {
            w = mul<T>(w, reinterpret_cast<const C<T>*>(a.sepx[j])[kx]);
            w = mul<T>(w, reinterpret_cast<const C<T>*>(a.sepy[j])[ky]);
            w = mul<T>(w, reinterpret_cast<const C<T>*>(a.sept[j])[kt]);
        }
    }
    if (a.conj_tab) w.y = -w.y;
    return w;
}

// One cyclic convolution of length N = R1 R2 per line, in place on x[r] (element t + R2 r
// of the line): DFT_N, product with B (conjugated when CONJB) plus add0 at frequency 0
// (thread t = 0), inverse DFT_N.  *a0 receives the DFT's zero frequency (thread t = 0).
// ex: the tile's LDS (row pitch W complex), free to be overwritten (every earlier read is
// before the barrier).
template <typename T, int R1, int R2, int W, bool CONJB>
__device__ __forceinline__ void rader_conv(C<T> (&x)[R1], const C<T>* bh, const C<T>* tw_f, const C<T>* tw_i, C<T>* ex,
                                           int q, int t, C<T> add0, C<T>* a0) {
    constexpr int CC = R1 / R2;
    RegDFT<R1, false, T>::run(x);
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1) x[k1] = mul<T>(x[k1], tw_f[k1 * R2 + t]);
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) ex[(k1 * R2 + t) * W + q] = x[k1];
    __syncthreads();
    C<T> v[CC][R2];
#pragma unroll
    for (int j = 0; j < CC; ++j) {
        const int k1 = CC * t + j;
#pragma unroll
        for (int tt = 0; tt < R2; ++tt) v[j][tt] = ex[(k1 * R2 + tt) * W + q];
        RegDFT<R2, false, T>::run(v[j]);
        if (j == 0 && t == 0) *a0 = v[0][0];
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) {
            C<T> b = bh[k1 + R1 * k2];
            if (CONJB) b.y = -b.y;
            v[j][k2] = mul<T>(v[j][k2], b);
        }
        if (j == 0 && t == 0) v[0][0] = add<T>(v[0][0], add0);
        RegDFT<R2, true, T>::run(v[j]);
#pragma unroll
        for (int tt = 1; tt < R2; ++tt) v[j][tt] = mulc<T>(v[j][tt], tw_i[tt * R1 + k1]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < CC; ++j)
#pragma unroll
        for (int tt = 0; tt < R2; ++tt) ex[((CC * t + j) * R2 + tt) * W + q] = v[j][tt];
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) x[k1] = ex[(k1 * R2 + t) * W + q];
    RegDFT<R1, true, T>::run(x);
}

template <typename T, int P, int MODE, bool ROWS>
__global__ void __launch_bounds__(kRaderW * RaderGeom<P>::R2) rader_pencil(PencilArgs a) {
    constexpr int R1 = RaderGeom<P>::R1, R2 = RaderGeom<P>::R2, N = P - 1, W = kRaderW, NT = W * R2;
    // LDS row pitch: rows (lines along x) are loaded point-fastest, so their tile rows are
    // padded by one complex value against bank conflicts
    constexpr int WP = ROWS ? W + 1 : W;
    static_assert(R1 * R2 == N && R1 % R2 == 0, "Rader geometry");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C<T>* tile = reinterpret_cast<C<T>*>(smem_raw);  // [P][WP], then the exchange buffer
    C<T>* tw_f = tile + P * WP;                         // [k1][t] = w_N^{t k1}
    C<T>* tw_i = tw_f + N;                              // [t][k1]
    C<T>* bh = tw_i + N;                                // B[k] = DFT_N(b)[k] / N
    C<T>* fl = bh + N;                                  // separable chains: prod_e T_e[k] along the line
    int* pin = reinterpret_cast<int*>(fl + P);            // g^q mod P
    int* pout = pin + N;                                  // g^-q mod P
    const int tid = threadIdx.x;
    const bool one_d = MODE == 0 && a.mul == 1;  // 1-D factor along the line only
    bool sep = MODE == 0;
    for (int j = 0; j < a.ntab; ++j) sep = sep && (one_d || a.tab3[j] == nullptr);
    if (sep) {
        const void* const* lt = one_d ? a.tab1 : (a.axis == 1 ? a.sepy : a.sept);
        for (int i = tid; i < P; i += NT) {
            C<T> v = mk<T>((T)1, (T)0);
            for (int j = 0; j < a.ntab; ++j) v = mul<T>(v, reinterpret_cast<const C<T>*>(lt[j])[i]);
            fl[i] = v;
        }
    }
    {
        // the plan's Rader block: w_N^j | B (forward) | B (inverse) | g^q | g^-q
        const C<T>* rt = reinterpret_cast<const C<T>*>(a.p.rtab);
        const int* ri = reinterpret_cast<const int*>(rt + 3 * N);
        for (int i = tid; i < N; i += NT) {
            const int k1 = i / R2, t = i - k1 * R2;
            const C<T> w = rt[t * k1];
            tw_f[k1 * R2 + t] = w;
            tw_i[t * R1 + k1] = w;
            bh[i] = rt[N + i];
            pin[i] = ri[i];
            pout[i] = ri[N + i];
        }
    }
    const long long plane = (long long)a.nx * a.ny;
    const int es = a.cplx ? 2 : 1;
    // element (point e, column c) of a tile at e * astride + c * cstride from its base:
    // rows: points along x, columns the y rows of one theta plane; pencils: points along
    // y (axis 1) or theta (axis 2), columns along x
    const long long astride = ROWS ? 1 : (a.axis == 1 ? (long long)a.nx : plane);
    const long long cstride = ROWS ? a.nx : 1;
    const int nother = ROWS ? a.m : (a.axis == 1 ? a.m : a.ny);
    const int ncol_tiles = (a.ncols + W - 1) / W;
    const int tiles_per_item = ncol_tiles * nother;
    const int ntiles = tiles_per_item * a.nitems;
    const int q = tid % W, t = tid / W;
    for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        const int u = xcd_contiguous(tl, ntiles);
        const int item = u / tiles_per_item;
        const int rem = u - item * tiles_per_item;
        const int other = rem / ncol_tiles;
        const int c0 = (rem - other * ncol_tiles) * W;
        const bool last_odd = (a.lone_in1 != nullptr || a.lone_out1 != nullptr) && item == a.nitems - 1;
        const long long obase =
            (ROWS || a.axis == 1 ? (long long)other * plane : (long long)other * a.nx) + (long long)c0 * cstride;
        const T* in0 = reinterpret_cast<const T*>(a.in0) + (long long)item * a.item_stride_in + obase * es;
        const T* in1 = last_odd ? reinterpret_cast<const T*>(a.lone_in1)
                                    : (a.in1 ? reinterpret_cast<const T*>(a.in1) + (long long)item * a.item_stride_in
                                             : nullptr);
        if (in1) in1 += obase * es;
        const int ncols = min(W, a.ncols - c0);
        __syncthreads();  // the previous tile's stores have read the LDS tile
        // The tile's loads go out STG at a time before their LDS writes, so that STG HBM
        // round trips overlap: element by element, every load waited for the one before
        // (the write to LDS needs its value), eleven round trips in a row per thread at 101.
        // The loads are unconditional (out-of-tile elements read a clamped address and are
        // zeroed after the load): a load under a branch made the compiler wait for every
        // earlier load first.  Rows: consecutive threads along the points of a row
        // (contiguous in memory).  In-tile offsets are 32-bit (P * plane * 2 < 2^31 for
        // every supported grid).
        constexpr int LIT = (P * W + NT - 1) / NT;  // elements per thread
        // (FP64 x rows keep one at a time: 48 -> 55 us at 101 with six, against 26.5 -> 23.8
        // and 29.6 -> 28.1 us for the FP32 pencils and rows)
        constexpr int STG = (sizeof(T) == 8 && ROWS) ? 1 : (LIT < 6 ? LIT : 6);
        const int ast = (int)astride * es, cst = (int)cstride * es;
        const bool has1 = in1 != nullptr;
        const T* in1p = has1 ? in1 : in0;
#pragma unroll 1
        for (int k0 = 0; k0 < LIT; k0 += STG) {
            C<T> lv[STG];
#pragma unroll
            for (int k = 0; k < STG; ++k) {
                const int i = tid + (k0 + k) * NT;
                const int c = ROWS ? i / P : i % W;
                const int e = ROWS ? i - c * P : i / W;
                const bool ok = k0 + k < LIT && i < P * W && c < ncols;
                const int off = min(e, P - 1) * ast + min(c, ncols - 1) * cst;
                const T vx = in0[off], vy = in1p[off];
                lv[k] = mk<T>(ok ? vx : (T)0, (ok && has1) ? vy : (T)0);
            }
#pragma unroll
            for (int k = 0; k < STG; ++k) {
                const int i = tid + (k0 + k) * NT;
                const int c = ROWS ? i / P : i % W;
                const int e = ROWS ? i - c * P : i / W;
                if (k0 + k < LIT && i < P * W) tile[e * WP + c] = lv[k];
            }
        }
        __syncthreads();
        C<T> x[R1];
        C<T> h0 = mk<T>((T)0, (T)0);  // X[0] or Y[0] (valid in thread t = 0)
        C<T> a0 = mk<T>((T)0, (T)0);
        if constexpr (MODE != 2) {
            const C<T> x0 = tile[q];
#pragma unroll
            for (int r = 0; r < R1; ++r) x[r] = tile[pin[t + R2 * r] * WP + q];
            rader_conv<T, R1, R2, WP, false>(x, bh, tw_f, tw_i, tile, q, t, x0, &a0);
            h0 = add<T>(x0, a0);  // X[0] = x[0] + sum_q a_q
            if constexpr (MODE == 0) {
                const int kx = min(c0 + q, a.ncols - 1);  // columns past the edge compute, unstored
                if (sep) {
                    // scale x the factors of x and of the outer coordinate (3-D product),
                    // then the line's from LDS
                    C<T> c = mk<T>((T)a.scale, (T)0);
                    const void* const* ot = a.axis == 1 ? a.sept : a.sepy;
                    for (int j = 0; j < a.ntab && !one_d; ++j) {
                        c = mul<T>(c, reinterpret_cast<const C<T>*>(a.sepx[j])[kx]);
                        c = mul<T>(c, reinterpret_cast<const C<T>*>(ot[j])[other]);
                    }
                    const T sg = a.conj_tab ? (T)-1 : (T)1;
#pragma unroll
                    for (int r = 0; r < R1; ++r) {
                        C<T> f = mul<T>(c, fl[pout[t + R2 * r]]);
                        f.y *= sg;
                        x[r] = mul<T>(x[r], f);
                    }
                    C<T> f0 = mul<T>(c, fl[0]);
                    f0.y *= sg;
                    h0 = mul<T>(h0, f0);
                } else {
#pragma unroll
                    for (int r = 0; r < R1; ++r) {
                        const int k = pout[t + R2 * r];
                        x[r] = mul<T>(x[r],
                                          rader_chain_factor<T>(a, kx, a.axis == 1 ? k : other, a.axis == 1 ? other : k));
                    }
                    h0 = mul<T>(h0, rader_chain_factor<T>(a, kx, a.axis == 1 ? 0 : other, a.axis == 1 ? other : 0));
                }
            }
        } else {
            h0 = tile[q];
#pragma unroll
            for (int r = 0; r < R1; ++r) x[r] = tile[pout[t + R2 * r] * WP + q];
        }
        if constexpr (MODE != 1) {
            rader_conv<T, R1, R2, WP, true>(x, bh, tw_f, tw_i, tile, q, t, h0, &a0);
            h0 = add<T>(h0, a0);  // y[0] = Y[0] + sum_m Y'[m]
        }
        __syncthreads();  // every exchange read is done: the tile takes the natural order
        const int* dst = MODE == 1 ? pout : pin;
#pragma unroll
        for (int r = 0; r < R1; ++r) tile[dst[t + R2 * r] * WP + q] = x[r];
        if (t == 0) tile[q] = h0;
        __syncthreads();
        T* out0 = reinterpret_cast<T*>(a.out0) + (long long)item * a.item_stride_out + obase * es;
        T* out1 = last_odd ? reinterpret_cast<T*>(a.lone_out1)
                               : (a.out1 ? reinterpret_cast<T*>(a.out1) + (long long)item * a.item_stride_out
                                         : nullptr);
        if (out1) out1 += obase * es;
        for (int i = tid; i < P * W; i += NT) {
            const int c = ROWS ? i / P : i % W;
            const int e = ROWS ? i - c * P : i / W;
            if (c < ncols) {
                const long long off = (e * astride + c * cstride) * es;
                const C<T> v = tile[e * WP + c];
                out0[off] = v.x;
                if (out1) out1[off] = v.y;
            }
        }
    }
}

bool rader_fast_supported(int L, bool dbl) {
    switch (L) {
        case 13: case 17: case 19: case 29: case 37: case 41: case 101:
            return true;
        case 61: case 73: case 97: case 109: case 113:
            return !dbl;
        default:
            return false;
    }
}

template <typename T, int P, int MODE, bool ROWS>
static hipError_t launch_rader_t(const PencilArgs& a, hipStream_t s) {
    const int ncol_tiles = (a.ncols + kRaderW - 1) / kRaderW;
    const long long ntiles = (long long)ncol_tiles * (ROWS || a.axis == 1 ? a.m : a.ny) * a.nitems;
    const int nb = (int)(ntiles < (1 << 20) ? ntiles : (1 << 20));
    constexpr size_t lds = rader_lds<T, P, ROWS>();
    hipLaunchKernelGGL((rader_pencil<T, P, MODE, ROWS>), dim3(nb), dim3(kRaderW * RaderGeom<P>::R2), lds, s, a);
    return hipGetLastError();
}

template <typename T, int P>
static hipError_t launch_rader_p(const PencilArgs& a, int mode, hipStream_t s) {
    if (a.axis == 0) {  // x rows
        if (mode == 0) return launch_rader_t<T, P, 0, true>(a, s);
        if (mode == 1) return launch_rader_t<T, P, 1, true>(a, s);
        if (mode == 2) return launch_rader_t<T, P, 2, true>(a, s);
        return hipErrorInvalidValue;
    }
    if (mode == 0) return launch_rader_t<T, P, 0, false>(a, s);
    if (mode == 1) return launch_rader_t<T, P, 1, false>(a, s);
    return launch_rader_t<T, P, 2, false>(a, s);
}

template <typename T>
static hipError_t launch_rader_typed(const PencilArgs& a, int mode, hipStream_t s) {
    switch (a.p.L) {
        case 13: return launch_rader_p<T, 13>(a, mode, s);
        case 17: return launch_rader_p<T, 17>(a, mode, s);
        case 19: return launch_rader_p<T, 19>(a, mode, s);
        case 29: return launch_rader_p<T, 29>(a, mode, s);
        case 37: return launch_rader_p<T, 37>(a, mode, s);
        case 41: return launch_rader_p<T, 41>(a, mode, s);
        case 101: return launch_rader_p<T, 101>(a, mode, s);
        default: break;
    }
    if constexpr (std::is_same<T, float>::value) {
        // FP32 only: in FP64 the R1 = 24..36 values per thread of these need 260-370 VGPRs
        switch (a.p.L) {
            case 61: return launch_rader_p<T, 61>(a, mode, s);
            case 73: return launch_rader_p<T, 73>(a, mode, s);
            case 97: return launch_rader_p<T, 97>(a, mode, s);
            case 109: return launch_rader_p<T, 109>(a, mode, s);
            case 113: return launch_rader_p<T, 113>(a, mode, s);
            default: break;
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_rader_pencil(const PencilArgs& a, bool dbl, hipStream_t s) {
    int mode;
    if (a.fwd && a.inv && (a.mul == 2 || a.mul == 1)) mode = 0;
    else if (a.fwd && !a.inv && a.mul == 0) mode = 1;
    else if (!a.fwd && a.inv && a.mul == 0) mode = 2;
    else return hipErrorInvalidValue;
    if (a.mode != 1 || a.items || (a.axis == 0 && a.mul == 2)) return hipErrorInvalidValue;
    return dbl ? launch_rader_typed<double>(a, mode, s) : launch_rader_typed<float>(a, mode, s);
}

}  // namespace se2c
