// Register-resident FP32 pass kernels for separable kernel tables
// (rho^[k; L] = Tx[k1] Ty[k2] Tt[k3], e.g. Gaussian x von Mises chains).
//
// The separable product commutes with transforms along the other axes, so the
// convolution factorises into 1-D circular convolutions along x, y and theta
// (each: DFT, product with the 1-D factor, inverse DFT; the 3-D DFT of eq.
// (3DFT) is the composition of the three 1-D DFTs).  Two passes over HBM when
// an x-theta slab fits in LDS, three otherwise:
//
// xt_slab_fast<NX, M, TPC>  one block per y-pair (rows 2s, 2s+1 packed as re/im):
//   1. load the pair in row layout: thread (g, t) holds x = t + R2 r (r < 16) of
//      rows theta = g + G i;
//   2. x convolution as a 16 x R2 decomposition: radix-16 DFT in registers,
//      twiddles w_NX^{t k1}, one LDS exchange (XOR-swizzled, bank-conflict
//      free), radix-R2 DFT, product with Tx/NX, and the mirror-image inverse;
//   3. transpose rows -> columns through LDS in chunks of 32 rows;
//   4. theta convolution of a whole column in registers (TPC = 2: the column is
//      split over a lane pair, and the radix-2 step, product and inverse step
//      are one 2 x 2 matrix per frequency);
//   5. store columns (each wave writes 1 KB contiguous per theta row).
//   Every input and output byte is touched once, so the pass streams with
//   nontemporal loads and stores (measured faster for this pass and for the
//   y pass that reads its output).
// line_pencil_fast<L>  16 adjacent x-pairs (float2 columns) x L points along y or
//   theta: the same R1 x R2 scheme (R1 = 16, or 32 for L = 512), product with
//   Ty/NY or Tt/M; persistent, with the next tile's loads issued early.
// x_rows_fast<NX>  three-pass schedule: the slab's x convolution alone on 16
//   theta-rows of one y-pair per block (NX up to 512).
#include "fast_common.hpp"
#include "regfft.hpp"
#include "sep_fast.hpp"

namespace se2c {

// Slab geometry.  TPC = threads per theta column in the column phase (1: the whole
// column in one thread; 2: even/odd theta split over neighbouring lanes).  The x phase
// splits a row into R1 values per thread x R2 lanes (R1 = 16; R1 = NX / 4 for
// NX = 3 * 2^k) and processes G rows at a time (G the largest power of two that fits
// the workgroup and a transpose chunk); for NX = 3 * 2^k the remaining lanes (whole
// wavefronts) idle during the x phase.
constexpr int pow2_floor(int v) { return v >= 32 ? 32 : v >= 16 ? 16 : v >= 8 ? 8 : v >= 4 ? 4 : v >= 2 ? 2 : 1; }

template <int NX, int M, int RCX = (M < 32 ? M : 32)> struct SlabGeom {
    static constexpr int TPC = M == 64 ? 2 : 1;
    static constexpr int NT = NX * TPC;
    static constexpr int R1 = (NX % 3 == 0) ? NX / 4 : 16;
    static constexpr int R2 = NX / R1;
    static constexpr int CC = R1 / R2;
    static constexpr int RC = RCX;                     // rows per transpose chunk
    static constexpr int H = M / RC;
    static constexpr int G = pow2_floor(NT / R2 < RC ? NT / R2 : RC);  // rows per x round
    static constexpr int RPT = M / G;                  // theta rows per thread in row layout
    static constexpr int XT = G * R2;                  // lanes of the x phase
    // LDS row pitch (complex): rows g and g + 1 start half a 64-bank cycle apart, so the
    // two row groups of a half-wave never share a bank
    static constexpr int P = NX + (R2 == 16 ? 16 : R2 % 16);
    static constexpr int MV = M / TPC;                 // theta values per thread in column layout
    static constexpr size_t LDS = sizeof(float2) * ((size_t)RC * P + 3 * NX + 2 * M);
    static_assert(R1 * R2 == NX && CC * R2 == R1 && M % G == 0 && M % RC == 0 && XT <= NT && XT % 16 == 0,
                  "slab geometry");
};

// One y-pair slab (rows 2s and 2s+1 of field `item`, packed as re/im) by the NT threads
// tid = 0 .. NT-1 of a workgroup, in the LDS region smem of Gm::LDS bytes.  Threads of a
// slab that is not `active` (the tail of a multi-class launch, or lanes beyond the last
// slab of a workgroup) take part in every barrier with the others but read and write no
// global memory and write no LDS; their LDS reads stay inside smem.
// ACC: the fields are always items (a.items) and their tables are read through an
// accessor (the multi-class launches); otherwise a.items may be null (then the launch's
// fields are a.in / a.out with one chain in the argument block) and the chain's table
// pointers are copied into a local array.
// CLAMPED: every thread belongs to a slab that names a valid one (a slab past its class's
// end repeats the class's last slab and writes the same values), so no load, LDS write
// or store needs a predicate.  The predicates of the general form cost the multi-class
// kernel about 90 VGPRs (244 against 156 for the 32 x 64 class alone).
template <int NX, int M, int RCX, bool ACC, bool CLAMPED = false>
__device__ __forceinline__ void slab_body(const FastSepArgs& a, int ny, int item, int s, bool active, int tid,
                                          unsigned char* smem) {
    using Gm = SlabGeom<NX, M, RCX>;
    constexpr int TPC = Gm::TPC, NT = Gm::NT, R1 = Gm::R1, R2 = Gm::R2, CC = Gm::CC, G = Gm::G, RPT = Gm::RPT,
                  RC = Gm::RC, H = Gm::H, P = Gm::P, MV = Gm::MV, XT = Gm::XT;
    float2* buf = reinterpret_cast<float2*>(smem);       // RC x P
    float2* tw_f = buf + RC * P;                         // [k1][t] = w_NX^{t k1}
    float2* tw_i = tw_f + NX;                            // [t][k1]
    float2* fx = tw_i + NX;                              // Tx / NX
    float2* ft = fx + NX;                                // Tt / M (TPC == 1)
    float4* cm = reinterpret_cast<float4*>(ft);          // [hh][k] = (S_k, E_hh,k) (TPC == 2)

    const long long plane = (long long)NX * ny;
    const int pl = (int)plane;
    // the field's input, output and table chain (shared by the launch, or per item)
    const float* fin = nullptr;
    float* fout = nullptr;
    const SepItem* it = a.items + item;
    // the chain's x and theta factors (a SEPARABLE table is Tx | Ty | Tt)
    const void* tx[SE2C_MAX_TABLES];
    const void* tt[SE2C_MAX_TABLES];
    int ntab = 0;
    if constexpr (!ACC) {
        if (!active) {
        } else if (a.items) {
            fin = reinterpret_cast<const float*>(it->in);
            fout = reinterpret_cast<float*>(it->out);
            ntab = it->ntab;
            for (int j = 0; j < ntab; ++j) {
                tx[j] = it->tab[j];
                tt[j] = reinterpret_cast<const float2*>(it->tab[j]) + NX + ny;
            }
        } else {
            fin = a.in + (long long)item * a.n;
            fout = a.out + (long long)item * a.n;
            ntab = a.ntab;
            for (int j = 0; j < ntab; ++j) {
                tx[j] = a.tx[j];
                tt[j] = a.tt[j];
            }
        }
    } else if (CLAMPED || active) {
        fin = reinterpret_cast<const float*>(it->in);
        fout = reinterpret_cast<float*>(it->out);
    }
    auto chain_x = [&](int i, float sc) {
        if constexpr (ACC)
            return chain_factor_of([&](int j) { return reinterpret_cast<const float2*>(it->tab[j]); }, it->ntab, i, sc,
                                   a.conj_tab);
        else
            return chain_factor(tx, ntab, i, sc, a.conj_tab);
    };
    auto chain_t = [&](int i, float sc) {
        if constexpr (ACC)
            return chain_factor_of([&](int j) { return reinterpret_cast<const float2*>(it->tab[j]) + NX + ny; },
                                   it->ntab, i, sc, a.conj_tab);
        else
            return chain_factor(tt, ntab, i, sc, a.conj_tab);
    };
    if (CLAMPED || active) {
        for (int i = tid; i < NX; i += NT) {
            const int k1 = i / R2, t = i - k1 * R2;
            const float2 w = a.tw[t * k1];
            tw_f[k1 * R2 + t] = w;
            tw_i[t * R1 + k1] = w;
        }
        for (int i = tid; i < NX; i += NT) fx[i] = chain_x(i, 1.0f / NX);
        if constexpr (TPC == 1) {
            for (int i = tid; i < M; i += NT) ft[i] = chain_t(i, 1.0f / M);
        } else {
            // the radix-2 step across the lane pair, the product with Tt and the inverse
            // radix-2 step fold into one 2 x 2 matrix per k < M/2 (see the column phase)
            for (int k = tid; k < MV; k += NT) {
                const float2 f0 = chain_t(k, 1.0f / M);
                const float2 f1 = chain_t(k + MV, 1.0f / M);
                const float2 sk = add<float>(f0, f1), dk = sub<float>(f0, f1);
                const float2 b = a.twt[k];  // w_M^k
                const float2 e0 = mul<float>(b, dk), e1 = mulc<float>(dk, b);
                cm[k] = make_float4(sk.x, sk.y, e0.x, e0.y);
                cm[MV + k] = make_float4(sk.x, sk.y, e1.x, e1.y);
            }
        }
    }
    __syncthreads();

    const int t = tid % R2, g = tid / R2;
    const bool xlane = XT == NT || tid < XT;   // takes part in the x phase (lanes from XT on idle)
    const bool xw = xlane && (CLAMPED || active);  // ... and loads and writes LDS
    // uniform tile base; per-lane offsets stay 32-bit (Nx Ny M < 2^30 is checked on the host)
    const float* __restrict__ in0 = fin + (long long)(2 * s) * NX;
    const float* __restrict__ in1 = in0 + NX;

    // 1. row-layout loads: rows theta = g + G i, columns x = t + R2 r
    float2 w[RPT][R1];
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int r = 0; r < R1; ++r) w[i][r] = make_float2(0.f, 0.f);
    if (xw) {
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
#pragma unroll
            for (int r = 0; r < R1; ++r) {
                const int off = (g + G * i) * pl + t + R2 * r;
                w[i][r] = make_float2(__builtin_nontemporal_load(in0 + off), __builtin_nontemporal_load(in1 + off));
            }
        }
    }
    __builtin_amdgcn_s_setprio(0);
    // 2. x convolution (R1 x R2 decomposition)
    if (xlane) {
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            RegDFT<R1, false, float>::run(w[i]);
#pragma unroll
            for (int k1 = 1; k1 < R1; ++k1) w[i][k1] = mul<float>(w[i][k1], tw_f[k1 * R2 + t]);
        }
    }
    float2* row = buf + g * P;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        if (i > 0) __syncthreads();
        if (xw) {
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) row[xpos_line<R1, R2>(k1, t)] = w[i][k1];
        }
        __syncthreads();
        float2 u[CC][R2];
        if (xlane) {
#pragma unroll
            for (int j = 0; j < CC; ++j) {
                const int k1 = CC * t + j;
#pragma unroll
                for (int tt = 0; tt < R2; ++tt) u[j][tt] = row[xpos_line<R1, R2>(k1, tt)];
                RegDFT<R2, false, float>::run(u[j]);
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) u[j][k2] = mul<float>(u[j][k2], fx[k1 + R1 * k2]);
                RegDFT<R2, true, float>::run(u[j]);
#pragma unroll
                for (int tt = 1; tt < R2; ++tt) u[j][tt] = mulc<float>(u[j][tt], tw_i[tt * R1 + k1]);
            }
        }
        __syncthreads();
        if (xw) {
#pragma unroll
            for (int j = 0; j < CC; ++j) {
#pragma unroll
                for (int tt = 0; tt < R2; ++tt) row[xpos_line<R1, R2>(CC * t + j, tt)] = u[j][tt];
            }
        }
        __syncthreads();
        if (xlane) {
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) w[i][k1] = row[xpos_line<R1, R2>(k1, t)];
            RegDFT<R1, true, float>::run(w[i]);
        }
    }
    // 3. rows -> columns through LDS, RC rows at a time
    const int xc = TPC == 1 ? tid : (tid >> 1);   // column owned in column layout
    const int hh = TPC == 1 ? 0 : (tid & 1);      // theta parity (TPC == 2)
    float2 v[MV];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        __syncthreads();
        if (xw) {
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                if (G * i >= h * RC && G * i < (h + 1) * RC) {
#pragma unroll
                    for (int r = 0; r < R1; ++r) buf[(g + G * i - h * RC) * P + t + R2 * r] = w[i][r];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int l = h * RC / TPC; l < (h + 1) * RC / TPC; ++l) v[l] = buf[(TPC * l + hh - h * RC) * P + xc];
    }
    // 4. theta convolution in registers
    if constexpr (TPC == 1) {
        RegDFT<M, false, float>::run(v);
#pragma unroll
        for (int k = 0; k < M; ++k) v[k] = mul<float>(v[k], ft[k]);
        RegDFT<M, true, float>::run(v);
    } else {
        // theta = hh + 2 s.  With Y_h = DFT over s of lane h's values and b = w_M^k,
        // X[k] = Y_0 + b Y_1 and X[k + M/2] = Y_0 - b Y_1; after the product with
        // F = Tt / M the inputs of the two inverse DFTs over s are
        //   U_0 = S Y_0 + (b D) Y_1,   U_1 = (conj(b) D) Y_0 + S Y_1,
        // S = F[k] + F[k + M/2], D = F[k] - F[k + M/2]: each lane combines its own
        // value with its neighbour's (DPP swap) through two precomputed factors.
        RegDFT<MV, false, float>::run(v);
        const float4* cmh = cm + MV * hh;
#pragma unroll
        for (int k = 0; k < MV; ++k) {
            const float2 o = swap_lane1(v[k]);
            const float4 c = cmh[k];
            const float2 y = v[k];
            v[k].x = c.x * y.x - c.y * y.y + c.z * o.x - c.w * o.y;
            v[k].y = c.x * y.y + c.y * y.x + c.z * o.y + c.w * o.x;
        }
        RegDFT<MV, true, float>::run(v);
    }
    // 5. store columns (CLAMPED: a repeated slab stores the same bits as the slab it
    // repeats, in the same workgroup after the same barriers, so its stores need no
    // predicate either; a predicated store phase cost the multi-class kernel spills)
    if (!CLAMPED && !active) return;
    float* __restrict__ out0 = fout + (long long)(2 * s) * NX;
    float* __restrict__ out1 = out0 + NX;
    __builtin_amdgcn_s_setprio(2);
#pragma unroll
    for (int l = 0; l < MV; ++l) {
        const int off = (TPC * l + hh) * pl + xc;
        __builtin_nontemporal_store(v[l].x, out0 + off);
        __builtin_nontemporal_store(v[l].y, out1 + off);
    }
}

template <int NX, int M>
__global__ void __launch_bounds__((SlabGeom<NX, M>::NT))
__attribute__((amdgpu_waves_per_eu(SlabGeom<NX, M>::NT >= 512 ? 4 : (SlabGeom<NX, M>::NT >= 256 ? 2 : 1))))
xt_slab_fast(FastSepArgs a) {
    // Wave priority: high while a wave issues its HBM loads and stores, low during the
    // arithmetic, so that a workgroup starting its memory phase is not held behind the
    // other workgroup's arithmetic on the same CU (measured 128 -> 118-122 us at
    // 256 x 256 x 64 x 16 fields).
    __builtin_amdgcn_s_setprio(2);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int nslab = a.ny / 2;
    const int item = blockIdx.x / nslab;  // one y-pair slab per block
    slab_body<NX, M, SlabGeom<NX, M>::RC, false>(a, a.ny, item, blockIdx.x - item * nslab, true, threadIdx.x, smem_raw);
}

// Line pencils: W = 16 adjacent x-pairs (float2 columns) x L points along y
// (axis 1) or theta (axis 2) at one outer coordinate (theta for y, y for theta).
// L = R1 x R2 with R1 = 16 values per thread (32 for L = 512).
// W = 16 adjacent x-pairs per tile (8 when the x-pair count is not a multiple of 16).
// L = 3 * 2^k lines use R1 = L / 4 values per thread (a mixed-radix register DFT).
template <int L, int WW> struct LineGeom {
    static constexpr int R1 = (L % 3 == 0) ? L / 4 : (L > 256 ? 32 : 16);
    static constexpr int R2 = L / R1;
    static constexpr int CC = R1 / R2;
    static constexpr int W = WW;
    static constexpr int NT = W * R2;
    static_assert(R1 * R2 == L && CC * R2 == R1, "line geometry");
};

template <int L, int WW>
__global__ void __launch_bounds__((LineGeom<L, WW>::NT)) line_pencil_fast(FastSepArgs a) {
    using Gm = LineGeom<L, WW>;
    constexpr int R1 = Gm::R1, R2 = Gm::R2, CC = Gm::CC, W = Gm::W, NT = Gm::NT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* buf = reinterpret_cast<float2*>(smem_raw);  // [k1*R2 + t][W]
    float2* tw_f = buf + L * W;                         // [k1][t] = w_L^{t k1}
    float2* tw_i = tw_f + L;                            // [t][k1]
    float2* fl = tw_i + L;                              // line factor / L
    const int tid = threadIdx.x;
    for (int i = tid; i < L; i += NT) {
        const int k1 = i / R2, t = i - k1 * R2;
        const float2 w = a.tw[t * k1];
        tw_f[k1 * R2 + t] = w;
        tw_i[t * R1 + k1] = w;
    }
    const int axis = a.axis;
    // offset of this axis' factor inside a SEPARABLE table (complex units)
    const int foff = axis == 1 ? a.nx : a.nx + a.ny;
    if (!a.items)
        for (int i = tid; i < L; i += NT)
            fl[i] = chain_factor(axis == 1 ? a.ty : a.tt, a.ntab, i, 1.0f / L, a.conj_tab);
    __syncthreads();

    const int q = tid % W, t = tid / W;
    const int ncols = a.nx / 2;
    const int ctiles = ncols / W;
    const int nouter = axis == 1 ? a.m : a.ny;
    // float2 strides: between points of a line, and between outer coordinates
    const int lstride = axis == 1 ? ncols : ncols * a.ny;
    const long long ostride = axis == 1 ? (long long)ncols * a.ny : (long long)ncols;
    const int per_item = ctiles * nouter;
    const int ntiles = per_item * a.nitems;
    auto tile_off = [&](int tile, int* item) -> long long {
        *item = tile / per_item;
        const int rem = tile - *item * per_item;
        const int o = rem / ctiles;
        const int ct = rem - o * ctiles;
        return (long long)o * ostride + ct * W;
    };
    // with items the pencil runs in place on each field's output (written by the previous pass)
    auto tile_src = [&](int tile) -> const float2* {
        int item;
        const long long off = tile_off(tile, &item);
        const float* base = a.items ? reinterpret_cast<const float*>(a.items[item].out) : a.in + (long long)item * a.n;
        return reinterpret_cast<const float2*>(base) + off;
    };
    auto tile_dst = [&](int tile) -> float2* {
        int item;
        const long long off = tile_off(tile, &item);
        float* base = a.items ? reinterpret_cast<float*>(a.items[item].out) : a.out + (long long)item * a.n;
        return reinterpret_cast<float2*>(base) + off;
    };
    // persistent blocks: the next tile's loads are issued before this tile's arithmetic
    const int lane_off = q + t * lstride;
    const int rstride = R2 * lstride;
    float2 nxt[R1];
    int tile = blockIdx.x;
    if (tile < ntiles) {
        const float2* src = tile_src(tile);
#pragma unroll
        for (int r = 0; r < R1; ++r) nxt[r] = (src + r * rstride)[lane_off];
    }
    int cur_item = -1;
    for (; tile < ntiles; tile += gridDim.x) {
        float2 w[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r) w[r] = nxt[r];
        const int next = tile + gridDim.x;
        if (next < ntiles) {
            // high wave priority while the next tile's loads are issued (as in the slab pass)
            const float2* src = tile_src(next);
#pragma unroll
            for (int r = 0; r < R1; ++r) nxt[r] = (src + r * rstride)[lane_off];
        }
        if (a.items) {
            const int item = tile / per_item;  // uniform across the block
            if (item != cur_item) {
                __syncthreads();
                const SepItem& it = a.items[item];
                const void* tl[SE2C_MAX_TABLES];
                for (int j = 0; j < it.ntab; ++j) tl[j] = reinterpret_cast<const float2*>(it.tab[j]) + foff;
                for (int i = tid; i < L; i += NT) fl[i] = chain_factor(tl, it.ntab, i, 1.0f / L, a.conj_tab);
                __syncthreads();
                cur_item = item;
            }
        }
        RegDFT<R1, false, float>::run(w);
#pragma unroll
        for (int k1 = 1; k1 < R1; ++k1) w[k1] = mul<float>(w[k1], tw_f[k1 * R2 + t]);
        __syncthreads();
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) buf[(k1 * R2 + t) * W + q] = w[k1];
        __syncthreads();
        float2 u[CC][R2];
#pragma unroll
        for (int j = 0; j < CC; ++j) {
            const int k1 = CC * t + j;
#pragma unroll
            for (int tt = 0; tt < R2; ++tt) u[j][tt] = buf[(k1 * R2 + tt) * W + q];
            RegDFT<R2, false, float>::run(u[j]);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) u[j][k2] = mul<float>(u[j][k2], fl[k1 + R1 * k2]);
            RegDFT<R2, true, float>::run(u[j]);
#pragma unroll
            for (int tt = 1; tt < R2; ++tt) u[j][tt] = mulc<float>(u[j][tt], tw_i[tt * R1 + k1]);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CC; ++j) {
#pragma unroll
            for (int tt = 0; tt < R2; ++tt) buf[((CC * t + j) * R2 + tt) * W + q] = u[j][tt];
        }
        __syncthreads();
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) w[k1] = buf[(k1 * R2 + t) * W + q];
        RegDFT<R1, true, float>::run(w);
        float2* dst = tile_dst(tile);
#pragma unroll
        for (int r = 0; r < R1; ++r) (dst + r * rstride)[lane_off] = w[r];
    }
}

// x rows: one block per (y-pair, 16 theta rows); rows 2s and 2s+1 of a field are
// packed as re/im, each row is convolved along x (the slab's x phase, R1 = 16 or 32
// values per thread) and written back.  Used when the x-theta slab does not fit in LDS.
template <int NX> struct RowGeom {
    static constexpr int R1 = NX > 256 ? 32 : 16;
    static constexpr int R2 = NX / R1;
    static constexpr int CC = R1 / R2;
    static constexpr int G = 16;                      // theta rows per tile
    static constexpr int NT = G * R2;
    static constexpr int P = NX + (R2 == 16 ? 16 : R2 % 16);  // LDS row pitch (complex)
};

template <int NX>
__global__ void __launch_bounds__(RowGeom<NX>::NT) x_rows_fast(FastSepArgs a) {
    using Gm = RowGeom<NX>;
    constexpr int R1 = Gm::R1, R2 = Gm::R2, CC = Gm::CC, G = Gm::G, NT = Gm::NT, P = Gm::P;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* buf = reinterpret_cast<float2*>(smem_raw);  // G x P
    float2* tw_f = buf + G * P;                          // [k1][t] = w_NX^{t k1}
    float2* tw_i = tw_f + NX;                            // [t][k1]
    float2* fx = tw_i + NX;                              // Tx / NX
    const int tid = threadIdx.x;
    const int nslab = a.ny / 2;
    const int trows = a.m / G;
    const int per_item = nslab * trows;
    const int tile = blockIdx.x;
    const int item = tile / per_item;
    const int rem = tile - item * per_item;
    const int tr = rem / nslab;
    const int s = rem - tr * nslab;
    const float* fin;
    float* fout;
    const void* tx[SE2C_MAX_TABLES];
    int ntab;
    if (a.items) {
        const SepItem& it = a.items[item];
        fin = reinterpret_cast<const float*>(it.in);
        fout = reinterpret_cast<float*>(it.out);
        ntab = it.ntab;
        for (int j = 0; j < ntab; ++j) tx[j] = it.tab[j];
    } else {
        fin = a.in + (long long)item * a.n;
        fout = a.out + (long long)item * a.n;
        ntab = a.ntab;
        for (int j = 0; j < ntab; ++j) tx[j] = a.tx[j];
    }
    for (int i = tid; i < NX; i += NT) {
        const int k1 = i / R2, t = i - k1 * R2;
        const float2 w = a.tw[t * k1];
        tw_f[k1 * R2 + t] = w;
        tw_i[t * R1 + k1] = w;
        fx[i] = chain_factor(tx, ntab, i, 1.0f / NX, a.conj_tab);
    }
    __syncthreads();

    const int t = tid % R2, g = tid / R2;
    const int pl = NX * a.ny;
    const long long tbase = (long long)(tr * G) * pl + (long long)(2 * s) * NX;
    const float* __restrict__ in0 = fin + tbase;
    const float* __restrict__ in1 = in0 + NX;
    float2 w[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) {
        const int off = g * pl + t + R2 * r;
        // plain loads: with 64-byte row segments a streaming hint re-fetched the other
        // half of each line (1.32x the algorithmic read bytes, and slower)
        w[r] = make_float2(in0[off], in1[off]);
    }
    RegDFT<R1, false, float>::run(w);
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1) w[k1] = mul<float>(w[k1], tw_f[k1 * R2 + t]);
    float2* row = buf + g * P;
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) row[xpos_line<R1, R2>(k1, t)] = w[k1];
    __syncthreads();
    float2 u[CC][R2];
#pragma unroll
    for (int j = 0; j < CC; ++j) {
        const int k1 = CC * t + j;
#pragma unroll
        for (int tt = 0; tt < R2; ++tt) u[j][tt] = row[xpos_line<R1, R2>(k1, tt)];
        RegDFT<R2, false, float>::run(u[j]);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) u[j][k2] = mul<float>(u[j][k2], fx[k1 + R1 * k2]);
        RegDFT<R2, true, float>::run(u[j]);
#pragma unroll
        for (int tt = 1; tt < R2; ++tt) u[j][tt] = mulc<float>(u[j][tt], tw_i[tt * R1 + k1]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < CC; ++j) {
#pragma unroll
        for (int tt = 0; tt < R2; ++tt) row[xpos_line<R1, R2>(CC * t + j, tt)] = u[j][tt];
    }
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) w[k1] = row[xpos_line<R1, R2>(k1, t)];
    RegDFT<R1, true, float>::run(w);
    float* __restrict__ out0 = fout + tbase;
    float* __restrict__ out1 = out0 + NX;
#pragma unroll
    for (int r = 0; r < R1; ++r) {
        const int off = g * pl + t + R2 * r;
        __builtin_nontemporal_store(w[r].x, out0 + off);
        __builtin_nontemporal_store(w[r].y, out1 + off);
    }
}

// ------------------------------------------------- multi-class launches (uneven batches)
// One launch per pass and class kind covers every shape class of a heterogeneous
// submission: a workgroup takes S = (its threads) / NT slabs (or pencil tiles) of one class
// side by side, each in its own LDS region; the classes are laid end to end over the grid, so
// small classes no longer run alone.  The transpose chunk is 16 rows wherever the x
// rounds need no more, which keeps every class within about 45 KB of LDS per workgroup.
// NTH: threads per workgroup, 256 for classes of 2^k points and 192 for 3 x 2^k (48 and
// 96 points: 48, 96 or 192 threads per slab), so that the slabs cover every workgroup.
template <int NX> constexpr int multi_slab_threads() { return (NX & (NX - 1)) == 0 ? SE2C_MULTI_THREADS : 192; }

template <int NX, int M> struct MultiSlab {
    static constexpr int NTH = multi_slab_threads<NX>();
    static constexpr int NT0 = NX * (M == 64 ? 2 : 1);
    static constexpr int R20 = NX / ((NX % 3 == 0) ? NX / 4 : 16);
    static constexpr int RC = (M < 32 || NT0 / R20 <= 16) ? 16 : 32;
    using Gm = SlabGeom<NX, M, RC>;
    static constexpr int S = NTH / Gm::NT;
    static constexpr size_t REGION = (Gm::LDS + 15) / 16 * 16;
    static constexpr size_t LDS = REGION * S;
};

template <int NX, int M>
__device__ __forceinline__ void slab_class(const MultiArgs& m, const MultiClass& c, int lb, unsigned char* smem) {
    using MS = MultiSlab<NX, M>;
    constexpr int NT = MS::Gm::NT, S = MS::S;
    // the S slabs of a workgroup cover its threads exactly
    constexpr bool CLAMPED = S * NT == MS::NTH;
    const int sub_raw = threadIdx.x / NT;
    const int sub = sub_raw < S ? sub_raw : S - 1;   // lanes beyond S shadow the last slab
    const int tid = threadIdx.x - sub_raw * NT;
    const int nslab = c.ny / 2;
    const int nunits = c.nitems * nslab;
    const int unit_raw = lb * S + sub;
    const bool active = sub_raw < S && unit_raw < nunits;
    const int unit = CLAMPED ? min(unit_raw, nunits - 1) : unit_raw;
    const int item = (CLAMPED || active) ? unit / nslab : 0;
    FastSepArgs a{};
    a.items = m.items + c.item0;
    a.tw = c.tw;
    a.twt = c.twt;
    a.conj_tab = m.conj_tab;
    slab_body<NX, M, MS::RC, true, CLAMPED>(a, c.ny, item, unit - item * nslab, active, tid,
                                             smem + (size_t)sub * MS::REGION);
}

// The classes in two launches by register budget: NX a power of two (153 VGPRs, three
// waves per SIMD) and NX = 3 * 2^k (24 values per thread at 96 points, 192-thread
// workgroups).
#define SE2C_MULTI_SLABS_P2(X) \
    X(32, 16) X(32, 32) X(32, 64) X(64, 16) X(64, 32) X(64, 64) X(128, 16) X(128, 32) X(128, 64) X(256, 16) X(256, 32)
#define SE2C_MULTI_SLABS_P3(X) X(48, 16) X(48, 32) X(48, 64) X(96, 16) X(96, 32) X(96, 64)
#define SE2C_MULTI_SLABS(X) SE2C_MULTI_SLABS_P2(X) SE2C_MULTI_SLABS_P3(X)

__device__ __forceinline__ const MultiClass& multi_class_of(const MultiArgs& m, int* lb) {
    int ci = 0;
    for (int k = 1; k < m.nclass; ++k)
        if ((int)blockIdx.x >= m.c[k].first_block) ci = k;
    *lb = blockIdx.x - m.c[ci].first_block;
    return m.c[ci];
}

#define SE2C_X(NX_, M_) \
    case NX_ * 1024 + M_: slab_class<NX_, M_>(m, c, lb, smem_raw); break;

__global__ void __launch_bounds__(SE2C_MULTI_THREADS) __attribute__((amdgpu_waves_per_eu(3)))
xt_slab_multi(MultiArgs m) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __builtin_amdgcn_s_setprio(2);
    int lb;
    const MultiClass& c = multi_class_of(m, &lb);
    switch (c.code) {
        SE2C_MULTI_SLABS_P2(SE2C_X)
        default: break;
    }
}

__global__ void __launch_bounds__(192) xt_slab_multi3(MultiArgs m) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __builtin_amdgcn_s_setprio(2);
    int lb;
    const MultiClass& c = multi_class_of(m, &lb);
    switch (c.code) {
        SE2C_MULTI_SLABS_P3(SE2C_X)
        default: break;
    }
}
#undef SE2C_X

// One pencil tile (W adjacent x-pairs x L points along y at theta = o, columns from
// ct * W) of field `item`, in place on the item's output, by threads tid < NT.
// CLAMPED: as for the slabs, an inactive tile repeats a valid one and every predicate
// goes (108 VGPRs, four waves per SIMD, for lines of 2^k points; 153 before).
template <int L, int WW, bool CLAMPED = false>
__device__ __forceinline__ void pencil_tile(const FastSepArgs& a, int nx, int ny, int item, int o, int ct, bool active,
                                            int tid, unsigned char* smem) {
    using Gm = LineGeom<L, WW>;
    constexpr int R1 = Gm::R1, R2 = Gm::R2, CC = Gm::CC, W = Gm::W;
    float2* buf = reinterpret_cast<float2*>(smem);  // [k1*R2 + t][W]
    float2* tw_f = buf + L * W;                      // [k1][t] = w_L^{t k1}
    float2* tw_i = tw_f + L;                         // [t][k1]
    float2* fl = tw_i + L;                           // line factor / L
    const int ncols = nx / 2;
    const int q = tid % W, t = tid / W;
    float2* base = nullptr;
    if (CLAMPED || active) {
        const SepItem& it = a.items[item];
        base = reinterpret_cast<float2*>(it.out) + (long long)o * ncols * ny + ct * W;
        auto ty = [&](int j) { return reinterpret_cast<const float2*>(it.tab[j]) + nx; };
        for (int i = tid; i < L; i += Gm::NT) {
            const int k1 = i / R2, tt = i - k1 * R2;
            const float2 w = a.tw[tt * k1];
            tw_f[k1 * R2 + tt] = w;
            tw_i[tt * R1 + k1] = w;
            fl[i] = chain_factor_of(ty, it.ntab, i, 1.0f / L, a.conj_tab);
        }
    }
    const int lane_off = q + t * ncols;
    const int rstride = R2 * ncols;
    float2 w[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) w[r] = make_float2(0.f, 0.f);
    if (CLAMPED || active) {
#pragma unroll
        for (int r = 0; r < R1; ++r) w[r] = (base + r * rstride)[lane_off];
    }
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    RegDFT<R1, false, float>::run(w);
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1) w[k1] = mul<float>(w[k1], tw_f[k1 * R2 + t]);
    if (CLAMPED || active) {
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) buf[(k1 * R2 + t) * W + q] = w[k1];
    }
    __syncthreads();
    float2 u[CC][R2];
#pragma unroll
    for (int j = 0; j < CC; ++j) {
        const int k1 = CC * t + j;
#pragma unroll
        for (int tt = 0; tt < R2; ++tt) u[j][tt] = buf[(k1 * R2 + tt) * W + q];
        RegDFT<R2, false, float>::run(u[j]);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) u[j][k2] = mul<float>(u[j][k2], fl[k1 + R1 * k2]);
        RegDFT<R2, true, float>::run(u[j]);
#pragma unroll
        for (int tt = 1; tt < R2; ++tt) u[j][tt] = mulc<float>(u[j][tt], tw_i[tt * R1 + k1]);
    }
    __syncthreads();
    if (CLAMPED || active) {
#pragma unroll
        for (int j = 0; j < CC; ++j) {
#pragma unroll
            for (int tt = 0; tt < R2; ++tt) buf[((CC * t + j) * R2 + tt) * W + q] = u[j][tt];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) w[k1] = buf[(k1 * R2 + t) * W + q];
    RegDFT<R1, true, float>::run(w);
    if (!CLAMPED && !active) return;
    __builtin_amdgcn_s_setprio(2);
#pragma unroll
    for (int r = 0; r < R1; ++r) (base + r * rstride)[lane_off] = w[r];
}

template <int L, int WW> struct MultiPencil {
    using Gm = LineGeom<L, WW>;
    static constexpr int S = SE2C_MULTI_THREADS / Gm::NT;
    static constexpr size_t REGION = (sizeof(float2) * ((size_t)L * WW + 3 * L) + 15) / 16 * 16;
    static constexpr size_t LDS = REGION * S;
};

template <int L, int WW>
__device__ __forceinline__ void pencil_class(const MultiArgs& m, const MultiClass& c, int lb, unsigned char* smem) {
    using MP = MultiPencil<L, WW>;
    constexpr int NT = MP::Gm::NT, S = MP::S;
    const int sub_raw = threadIdx.x / NT;
    const int sub = sub_raw < S ? sub_raw : S - 1;
    const int tid = threadIdx.x - sub_raw * NT;
    const int ctiles = (c.nx / 2) / WW;
    const int per_item = ctiles * c.m;
    // every class's tiles cover the workgroup's threads exactly (NT divides 256); a tile
    // past the class's end repeats the class's last tile, in the same workgroup
    constexpr bool CLAMPED = S * NT == SE2C_MULTI_THREADS;
    const int nunits = c.nitems * per_item;
    const int unit_raw = lb * S + sub;
    const bool active = sub_raw < S && unit_raw < nunits;
    const int unit = CLAMPED ? min(unit_raw, nunits - 1) : unit_raw;
    const int item = (CLAMPED || active) ? unit / per_item : 0;
    const int rem = unit - item * per_item;
    const int o = rem / ctiles;
    FastSepArgs a{};
    a.items = m.items + c.item0;
    a.tw = c.tw;
    a.conj_tab = m.conj_tab;
    pencil_tile<L, WW, CLAMPED>(a, c.nx, c.ny, item, o, rem - o * ctiles, active, tid,
                                smem + (size_t)sub * MP::REGION);
}

// Pencil classes in two launches as well: lines of 2^k points fit the 128 VGPRs of four
// waves per SIMD, the 96-point lines (24 values per thread) do not; 48 goes with 96, so
// that square problems of a class kind keep both passes in one kind.
#define SE2C_MULTI_PENCILS_A(X) \
    X(32, 16) X(32, 8) X(64, 16) X(64, 8) X(128, 16) X(128, 8) X(256, 16) X(256, 8)
#define SE2C_MULTI_PENCILS_B(X) X(48, 16) X(48, 8) X(96, 16) X(96, 8)
#define SE2C_MULTI_PENCILS(X) SE2C_MULTI_PENCILS_A(X) SE2C_MULTI_PENCILS_B(X)

#define SE2C_X(L_, W_) \
    case L_ * 1024 + W_: pencil_class<L_, W_>(m, c, lb, smem_raw); break;

__global__ void __launch_bounds__(SE2C_MULTI_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
y_pencil_multi(MultiArgs m) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __builtin_amdgcn_s_setprio(2);
    int lb;
    const MultiClass& c = multi_class_of(m, &lb);
    switch (c.code) {
        SE2C_MULTI_PENCILS_A(SE2C_X)
        default: break;
    }
}

__global__ void __launch_bounds__(SE2C_MULTI_THREADS) y_pencil_multi3(MultiArgs m) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __builtin_amdgcn_s_setprio(2);
    int lb;
    const MultiClass& c = multi_class_of(m, &lb);
    switch (c.code) {
        SE2C_MULTI_PENCILS_B(SE2C_X)
        default: break;
    }
}
#undef SE2C_X

// Host side of the multi-class launches: shape support, class codes, units per
// workgroup and LDS.
bool multi_slab_supported(int nx, int m) {
#define SE2C_X(NX_, M_) if (nx == NX_ && m == M_) return true;
    SE2C_MULTI_SLABS(SE2C_X)
#undef SE2C_X
    return false;
}

static int multi_slab_per_block(int nx, int m) {
#define SE2C_X(NX_, M_) if (nx == NX_ && m == M_) return MultiSlab<NX_, M_>::S;
    SE2C_MULTI_SLABS(SE2C_X)
#undef SE2C_X
    return 0;
}

static size_t multi_slab_lds(int nx, int m) {
#define SE2C_X(NX_, M_) if (nx == NX_ && m == M_) return MultiSlab<NX_, M_>::LDS;
    SE2C_MULTI_SLABS(SE2C_X)
#undef SE2C_X
    return 0;
}

static int pencil_w_for(int nx) { return (nx / 2) % 16 == 0 ? 16 : 8; }

bool multi_pencil_supported(int nx, int ny) {
    const int w = pencil_w_for(nx);
    if (nx % 16) return false;
#define SE2C_X(L_, W_) if (ny == L_ && w == W_) return true;
    SE2C_MULTI_PENCILS(SE2C_X)
#undef SE2C_X
    return false;
}

static int multi_pencil_per_block(int ny, int w) {
#define SE2C_X(L_, W_) if (ny == L_ && w == W_) return MultiPencil<L_, W_>::S;
    SE2C_MULTI_PENCILS(SE2C_X)
#undef SE2C_X
    return 0;
}

static size_t multi_pencil_lds(int ny, int w) {
#define SE2C_X(L_, W_) if (ny == L_ && w == W_) return MultiPencil<L_, W_>::LDS;
    SE2C_MULTI_PENCILS(SE2C_X)
#undef SE2C_X
    return 0;
}

// Fills the per-class launch fields (code, first workgroup) of one pass and returns the
// grid size and LDS; classes keep the caller's order.
static hipError_t plan_multi(MultiArgs& m, bool pencil, int* blocks, size_t* lds) {
    int first = 0;
    size_t l = 0;
    for (int k = 0; k < m.nclass; ++k) {
        MultiClass& c = m.c[k];
        int per, units;
        size_t cl;
        if (pencil) {
            const int w = pencil_w_for(c.nx);
            per = multi_pencil_per_block(c.ny, w);
            cl = multi_pencil_lds(c.ny, w);
            c.code = c.ny * 1024 + w;
            units = c.nitems * ((c.nx / 2) / w) * c.m;
            c.tw = c.twy;
        } else {
            per = multi_slab_per_block(c.nx, c.m);
            cl = multi_slab_lds(c.nx, c.m);
            c.code = c.nx * 1024 + c.m;
            units = c.nitems * (c.ny / 2);
            c.tw = c.twx;
        }
        if (per < 1) return hipErrorInvalidValue;
        c.first_block = first;
        first += (units + per - 1) / per;
        l = l > cl ? l : cl;
    }
    *blocks = first;
    *lds = l;
    return hipSuccess;
}

hipError_t launch_slab_multi(MultiArgs m, hipStream_t s) {
    // power-of-two classes first (most of the points), then the 3 * 2^k classes; each
    // launch keeps the classes' order (largest first)
    MultiArgs part[2] = {m, m};
    part[0].nclass = part[1].nclass = 0;
    for (int k = 0; k < m.nclass; ++k) {
        const int nx = m.c[k].nx;
        MultiArgs& q = part[(nx & (nx - 1)) == 0 ? 0 : 1];
        q.c[q.nclass++] = m.c[k];
    }
    for (int h = 0; h < 2; ++h) {
        if (part[h].nclass == 0) continue;
        int blocks = 0;
        size_t lds = 0;
        hipError_t e = plan_multi(part[h], false, &blocks, &lds);
        if (e != hipSuccess) return e;
        if (h == 0) hipLaunchKernelGGL(xt_slab_multi, dim3(blocks), dim3(SE2C_MULTI_THREADS), lds, s, part[h]);
        else hipLaunchKernelGGL(xt_slab_multi3, dim3(blocks), dim3(192), lds, s, part[h]);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_pencil_multi(MultiArgs m, hipStream_t s) {
    MultiArgs part[2] = {m, m};
    part[0].nclass = part[1].nclass = 0;
    for (int k = 0; k < m.nclass; ++k) {
        const int ny = m.c[k].ny;
        MultiArgs& q = part[(ny & (ny - 1)) == 0 ? 0 : 1];
        q.c[q.nclass++] = m.c[k];
    }
    for (int h = 0; h < 2; ++h) {
        if (part[h].nclass == 0) continue;
        int blocks = 0;
        size_t lds = 0;
        hipError_t e = plan_multi(part[h], true, &blocks, &lds);
        if (e != hipSuccess) return e;
        if (h == 0) hipLaunchKernelGGL(y_pencil_multi, dim3(blocks), dim3(SE2C_MULTI_THREADS), lds, s, part[h]);
        else hipLaunchKernelGGL(y_pencil_multi3, dim3(blocks), dim3(SE2C_MULTI_THREADS), lds, s, part[h]);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------------------ dispatch
template <int NX, int M>
static size_t slab_fast_lds() {
    return SlabGeom<NX, M>::LDS;
}

template <int L, int W>
static size_t pencil_fast_lds() {
    return sizeof(float2) * ((size_t)L * W + 3 * L);
}

template <int NX>
static size_t rows_fast_lds() {
    return sizeof(float2) * ((size_t)RowGeom<NX>::G * RowGeom<NX>::P + 3 * NX);
}

template <int NX, int M>
static hipError_t launch_slab_fast_t(const FastSepArgs& a, int nblocks, hipStream_t s) {
    const size_t lds = slab_fast_lds<NX, M>();
    const int nthr = SlabGeom<NX, M>::NT;
    hipLaunchKernelGGL((xt_slab_fast<NX, M>), dim3(nblocks), dim3(nthr), lds, s, a);
    return hipGetLastError();
}

template <int L, int W>
static hipError_t launch_pencil_fast_t(const FastSepArgs& a, hipStream_t s) {
    const size_t lds = pencil_fast_lds<L, W>();
    const int nouter = a.axis == 1 ? a.m : a.ny;
    const int ntiles = (a.nx / 2 / W) * nouter * a.nitems;
    // persistent grid: a few blocks per CU (no more than fit at once), each walks its
    // share of tiles
    static const int fit = [lds] {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void*>(line_pencil_fast<L, W>),
                                                         LineGeom<L, W>::NT, lds) != hipSuccess || b < 1)
            b = 1;
        return b;
    }();
    int nblocks = a.grid_blocks < a.cus * fit ? a.grid_blocks : a.cus * fit;
    if (ntiles < nblocks) nblocks = ntiles;
    const int nthr = LineGeom<L, W>::NT;
    hipLaunchKernelGGL((line_pencil_fast<L, W>), dim3(nblocks), dim3(nthr), lds, s, a);
    return hipGetLastError();
}

template <int L>
static hipError_t launch_pencil_w(const FastSepArgs& a, hipStream_t s) {
    return (a.nx / 2) % 16 == 0 ? launch_pencil_fast_t<L, 16>(a, s) : launch_pencil_fast_t<L, 8>(a, s);
}

template <int NX>
static hipError_t launch_rows_fast_t(const FastSepArgs& a, hipStream_t s) {
    const size_t lds = rows_fast_lds<NX>();
    const int nblocks = (a.ny / 2) * (a.m / RowGeom<NX>::G) * a.nitems;
    hipLaunchKernelGGL((x_rows_fast<NX>), dim3(nblocks), dim3(RowGeom<NX>::NT), lds, s, a);
    return hipGetLastError();
}

bool slab_fast_supported(int nx, int m) {
    return (nx == 32 || nx == 48 || nx == 64 || nx == 96 || nx == 128 || nx == 256) && (m == 16 || m == 32 || m == 64);
}

static bool line_len_ok(int l) {
    return l == 32 || l == 48 || l == 64 || l == 96 || l == 128 || l == 256 || l == 512;
}

// columns come in x-pairs, W = 16 or 8 of them per tile
bool pencil_fast_supported(int nx, int ny) { return line_len_ok(ny) && nx % 16 == 0; }

bool three_pass_fast_supported(int nx, int ny, int m) {
    return (nx == 64 || nx == 128 || nx == 256 || nx == 512) && line_len_ok(ny) && line_len_ok(m);
}

#define SE2C_SLAB_CASE(NX_, M_) \
    if (a.nx == NX_ && a.m == M_) return launch_slab_fast_t<NX_, M_>(a, nblocks, s);

hipError_t launch_slab_fast(const FastSepArgs& a, hipStream_t s) {
    const int nblocks = (a.ny / 2) * a.nitems;  // one block per y-pair slab
    SE2C_SLAB_CASE(32, 16) SE2C_SLAB_CASE(32, 32) SE2C_SLAB_CASE(32, 64)
    SE2C_SLAB_CASE(48, 16) SE2C_SLAB_CASE(48, 32) SE2C_SLAB_CASE(48, 64)
    SE2C_SLAB_CASE(96, 16) SE2C_SLAB_CASE(96, 32) SE2C_SLAB_CASE(96, 64)
    SE2C_SLAB_CASE(64, 16) SE2C_SLAB_CASE(64, 32) SE2C_SLAB_CASE(64, 64)
    SE2C_SLAB_CASE(128, 16) SE2C_SLAB_CASE(128, 32) SE2C_SLAB_CASE(128, 64)
    SE2C_SLAB_CASE(256, 16) SE2C_SLAB_CASE(256, 32) SE2C_SLAB_CASE(256, 64)
    return hipErrorInvalidValue;
}

hipError_t launch_pencil_fast(const FastSepArgs& a, hipStream_t s) {
    const int L = a.axis == 1 ? a.ny : a.m;
    if (L == 32) return launch_pencil_w<32>(a, s);
    if (L == 48) return launch_pencil_w<48>(a, s);
    if (L == 64) return launch_pencil_w<64>(a, s);
    if (L == 96) return launch_pencil_w<96>(a, s);
    if (L == 128) return launch_pencil_w<128>(a, s);
    if (L == 256) return launch_pencil_w<256>(a, s);
    if (L == 512) return launch_pencil_w<512>(a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_rows_fast(const FastSepArgs& a, hipStream_t s) {
    if (a.nx == 64) return launch_rows_fast_t<64>(a, s);
    if (a.nx == 128) return launch_rows_fast_t<128>(a, s);
    if (a.nx == 256) return launch_rows_fast_t<256>(a, s);
    if (a.nx == 512) return launch_rows_fast_t<512>(a, s);
    return hipErrorInvalidValue;
}

#define SE2C_SLAB_ATTR(NX_, M_)                                                                        \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(xt_slab_fast<NX_, M_>),                        \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)slab_fast_lds<NX_, M_>()); \
    if (e != hipSuccess) return e;

#define SE2C_PENCIL_ATTR(L_, W_)                                                                          \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(line_pencil_fast<L_, W_>),                       \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)pencil_fast_lds<L_, W_>());  \
    if (e != hipSuccess) return e;
#define SE2C_LINE_ATTR(L_) SE2C_PENCIL_ATTR(L_, 16) SE2C_PENCIL_ATTR(L_, 8)
#define SE2C_ROWS_ATTR(NX_)                                                                                \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(x_rows_fast<NX_>),                               \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)rows_fast_lds<NX_>());      \
    if (e != hipSuccess) return e;

hipError_t prepare_fast_kernels() {
    hipError_t e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(xt_slab_multi), hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(xt_slab_multi3), hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(y_pencil_multi), hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(y_pencil_multi3), hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    if (e != hipSuccess) return e;
    SE2C_SLAB_ATTR(32, 16) SE2C_SLAB_ATTR(32, 32) SE2C_SLAB_ATTR(32, 64)
    SE2C_SLAB_ATTR(48, 16) SE2C_SLAB_ATTR(48, 32) SE2C_SLAB_ATTR(48, 64)
    SE2C_SLAB_ATTR(96, 16) SE2C_SLAB_ATTR(96, 32) SE2C_SLAB_ATTR(96, 64)
    SE2C_SLAB_ATTR(64, 16) SE2C_SLAB_ATTR(64, 32) SE2C_SLAB_ATTR(64, 64)
    SE2C_SLAB_ATTR(128, 16) SE2C_SLAB_ATTR(128, 32) SE2C_SLAB_ATTR(128, 64)
    SE2C_SLAB_ATTR(256, 16) SE2C_SLAB_ATTR(256, 32) SE2C_SLAB_ATTR(256, 64)
    SE2C_LINE_ATTR(32) SE2C_LINE_ATTR(48) SE2C_LINE_ATTR(64) SE2C_LINE_ATTR(96) SE2C_LINE_ATTR(128)
    SE2C_LINE_ATTR(256) SE2C_LINE_ATTR(512)
    SE2C_ROWS_ATTR(64) SE2C_ROWS_ATTR(128) SE2C_ROWS_ATTR(256) SE2C_ROWS_ATTR(512)
    return hipSuccess;
}

}  // namespace se2c
