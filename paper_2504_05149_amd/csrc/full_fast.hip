// Register-resident FP32 kernels of the full-table path: out = S_K[f, rho] with an
// arbitrary (non-separable) coefficient table, i.e. out = iDFT3(W . DFT3(F) . T) / n
// (eqs. (FkLv), (SKfg), (3iDFT); the sign W and 1/n are folded into the table).
//
// Two real fields are transformed at once as z = f_a + i f_b: for a real-kernel table
// (T[-k] = conj T[k]) the inverse of T . Z^ has real part S_K[f_a] and imaginary part
// S_K[f_b].  Three passes over HBM:
//
// xt_full<NX, M, DIR = 0>  one block per (pair, y row): forward DFT along x (16 x R2
//   register decomposition, one XOR-swizzled LDS exchange), rows -> columns through
//   LDS, forward DFT along theta in registers (TPC = 2: the last radix-2 step across
//   neighbouring lanes via DPP); stores the x-theta spectrum as re/im planes.
// y_full<NY, MODE>  one block per (theta frequency, 16 or 32 x frequencies, pair), the
//   blocks of one tile back to back on one XCD: forward DFT along y, [copy of the
//   spectrum], product with the table, inverse DFT along y, in place; MODE 2 walks the
//   pairs in one block and accumulates the kernel-sample gradient of the batch (see below).
// xt_full<NX, M, DIR = 1>  the mirror image of the first pass: inverse DFT along
//   theta (columns), columns -> rows, inverse DFT along x, stores the two real fields.
// xt_full<NX, M, DIR = 2>  the first pass without the theta DFT (x spectrum at every
//   theta row), and y_full MODE 1 / MODE 4 (forward / inverse along y only): the passes
//   around a theta pass that needs theta in space (sums of SE(2)-shifted kernels).
#include "fast_common.hpp"
#include "full_fast.hpp"
#include "regfft.hpp"

namespace se2c {

template <int NX, int M> struct FullSlabGeom {
    static constexpr int TPC = M == 64 ? 2 : 1;      // threads per theta column
    static constexpr int NT = NX * TPC;
    static constexpr int R2 = NX / 16;               // second-stage radix along x
    static constexpr int CC = 16 / R2;               // first-stage frequencies per thread
    static constexpr int G = NT / R2;                // row groups in row layout
    static constexpr int RPT = M / G;                // theta rows per thread in row layout
    static constexpr int RC = M < 32 ? M : 32;       // rows per transpose chunk
    static constexpr int H = M / RC;
    static constexpr int P = NX + (R2 == 16 ? 16 : R2 % 16);  // LDS row pitch (complex)
    static constexpr int MV = M / TPC;               // theta values per thread in column layout
    static_assert(G <= RC && RPT >= 1 && M % G == 0, "tile geometry");
};

template <int NX, int M>
static constexpr size_t full_slab_lds() {
    using Gm = FullSlabGeom<NX, M>;
    return sizeof(float2) * ((size_t)Gm::RC * Gm::P + 2 * NX + M);
}

template <int NX, int M, int DIR>
__global__ void __launch_bounds__((FullSlabGeom<NX, M>::NT))
__attribute__((amdgpu_waves_per_eu(FullSlabGeom<NX, M>::NT >= 512 ? 4 : (FullSlabGeom<NX, M>::NT >= 256 ? 2 : 1))))
xt_full(FullFastArgs a) {
    using Gm = FullSlabGeom<NX, M>;
    constexpr int TPC = Gm::TPC, NT = Gm::NT, R2 = Gm::R2, CC = Gm::CC, G = Gm::G, RPT = Gm::RPT, RC = Gm::RC,
                  H = Gm::H, P = Gm::P, MV = Gm::MV;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* buf = reinterpret_cast<float2*>(smem_raw);  // RC x P
    float2* tw_f = buf + RC * P;                         // [k1][t] = w_NX^{t k1}
    float2* tw_i = tw_f + NX;                            // [t][k1]
    float2* twl = tw_i + NX;                             // TPC == 2: [h][k] = 1 (h = 0), w_M^k (h = 1)
    const int tid = threadIdx.x;
    for (int i = tid; i < NX; i += NT) {
        const int k1 = i / R2, t = i - k1 * R2;
        const float2 w = a.twx[t * k1];
        tw_f[k1 * R2 + t] = w;
        tw_i[t * 16 + k1] = w;
    }
    if (TPC == 2)
        for (int i = tid; i < M; i += NT) twl[i] = i < MV ? make_float2(1.f, 0.f) : a.twt[i - MV];
    __syncthreads();

    const int pair = blockIdx.x / a.ny;
    const int y = blockIdx.x - pair * a.ny;
    const int pl = NX * a.ny;
    const bool has_b = 2 * pair + 1 < a.batch;
    const int t = tid % R2, g = tid / R2;
    const int xc = TPC == 1 ? tid : (tid >> 1);
    const int hh = TPC == 1 ? 0 : (tid & 1);
    float2 w[RPT][16];
    float2 v[MV];

    if constexpr (DIR == 0 || DIR == 2) {
        // a lone last field is paired with zero (its row is read twice and masked, which
        // keeps the loads free of per-load branches)
        const float* __restrict__ in0 = a.in + (long long)(2 * pair) * a.n + (long long)y * NX;
        const float* __restrict__ in1 = has_b ? in0 + a.n : in0;
        const float im_mask = has_b ? 1.f : 0.f;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int off = (g + G * i) * pl + t + R2 * r;
                w[i][r] = make_float2(__builtin_nontemporal_load(in0 + off),
                                      im_mask * __builtin_nontemporal_load(in1 + off));
            }
        }
        // forward DFT along x of each row; afterwards w[i][j * R2 + k2] = X[k1 + 16 k2], k1 = CC t + j
        float2* row = buf + g * P;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            dft16<float, false>(w[i]);
#pragma unroll
            for (int k1 = 1; k1 < 16; ++k1) w[i][k1] = mul<float>(w[i][k1], tw_f[k1 * R2 + t]);
            if (i > 0) __syncthreads();
#pragma unroll
            for (int k1 = 0; k1 < 16; ++k1) row[xpos<R2>(k1, t)] = w[i][k1];
            __syncthreads();
#pragma unroll
            for (int j = 0; j < CC; ++j) {
                const int k1 = CC * t + j;
                float2 u[R2];
#pragma unroll
                for (int tt = 0; tt < R2; ++tt) u[tt] = row[xpos<R2>(k1, tt)];
                RegDFT<R2, false, float>::run(u);
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) w[i][j * R2 + k2] = u[k2];
            }
        }
        // rows -> columns (x frequency kx = xc in column layout)
#pragma unroll
        for (int h = 0; h < H; ++h) {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                if (G * i >= h * RC && G * i < (h + 1) * RC) {
#pragma unroll
                    for (int j = 0; j < CC; ++j)
#pragma unroll
                        for (int k2 = 0; k2 < R2; ++k2)
                            buf[(g + G * i - h * RC) * P + CC * t + j + 16 * k2] = w[i][j * R2 + k2];
                }
            }
            __syncthreads();
#pragma unroll
            for (int l = h * RC / TPC; l < (h + 1) * RC / TPC; ++l) v[l] = buf[(TPC * l + hh - h * RC) * P + xc];
        }
        // forward DFT along theta (DIR 2: x only, theta stays spatial)
        if constexpr (DIR == 2) {
        } else if constexpr (TPC == 1) {
            RegDFT<M, false, float>::run(v);
        } else {
            // theta = hh + 2 s: Y_hh = DFT over s; X[k] = Y_0 + w^k Y_1, X[k + M/2] = Y_0 - w^k Y_1
            // Lane h first multiplies its own value by twl[h][k] (1 or w^k); with o the
            // neighbour's product, lane 0 keeps b + o and lane 1 o - b (no divergent code).
            RegDFT<MV, false, float>::run(v);
            const float sg = hh ? -1.f : 1.f;
            const float2* twh = twl + hh * MV;
#pragma unroll
            for (int k = 0; k < MV; ++k) {
                const float2 b = mul<float>(v[k], twh[k]);
                const float2 o = swap_lane1(b);
                v[k] = make_float2(fmaf(sg, b.x, o.x), fmaf(sg, b.y, o.y));
            }
        }
        float* __restrict__ o_re = a.out + (long long)(2 * pair) * a.n + (long long)y * NX;
        float* __restrict__ o_im = (has_b ? a.out + (long long)(2 * pair + 1) * a.n : a.lone) + (long long)y * NX;
#pragma unroll
        for (int l = 0; l < MV; ++l) {
            // theta frequency (after the split of TPC == 2), or theta row TPC l + hh (DIR 2)
            const int kt = DIR == 2 ? TPC * l + hh : (TPC == 1 ? l : l + hh * MV);
            const int off = kt * pl + xc;
            __builtin_nontemporal_store(v[l].x, o_re + off);
            __builtin_nontemporal_store(v[l].y, o_im + off);
        }
    } else {
        const float* __restrict__ i_re = a.in + (long long)(2 * pair) * a.n + (long long)y * NX;
        const float* __restrict__ i_im =
            (has_b ? a.in + (long long)(2 * pair + 1) * a.n : a.lone) + (long long)y * NX;
#pragma unroll
        for (int l = 0; l < MV; ++l) {
            const int kt = TPC == 1 ? l : l + hh * MV;
            const int off = kt * pl + xc;
            v[l] = make_float2(__builtin_nontemporal_load(i_re + off), __builtin_nontemporal_load(i_im + off));
        }
        // inverse DFT along theta
        if constexpr (TPC == 1) {
            RegDFT<M, true, float>::run(v);
        } else {
            // lane 0 holds Z[k], lane 1 Z[k + M/2]: U_0 = Z[k] + Z[k + M/2],
            // U_1 = conj(w^k) (Z[k] - Z[k + M/2]); then inverse DFT over s gives theta = hh + 2 s
            // d = own sign + neighbour (lane 0: Z[k] + Z[k + M/2], lane 1: Z[k] - Z[k + M/2]),
            // then lane h multiplies by conj(twl[h][k]) (1 or conj(w^k))
            const float sg = hh ? -1.f : 1.f;
            const float2* twh = twl + hh * MV;
#pragma unroll
            for (int k = 0; k < MV; ++k) {
                const float2 o = swap_lane1(v[k]);
                const float2 d = make_float2(fmaf(sg, v[k].x, o.x), fmaf(sg, v[k].y, o.y));
                v[k] = mulc<float>(d, twh[k]);
            }
            RegDFT<MV, true, float>::run(v);
        }
        // columns -> rows (x frequencies in row layout: w[i][j * R2 + k2] = X[CC t + j + 16 k2])
#pragma unroll
        for (int h = 0; h < H; ++h) {
            __syncthreads();
#pragma unroll
            for (int l = h * RC / TPC; l < (h + 1) * RC / TPC; ++l) buf[(TPC * l + hh - h * RC) * P + xc] = v[l];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                if (G * i >= h * RC && G * i < (h + 1) * RC) {
#pragma unroll
                    for (int j = 0; j < CC; ++j)
#pragma unroll
                        for (int k2 = 0; k2 < R2; ++k2)
                            w[i][j * R2 + k2] = buf[(g + G * i - h * RC) * P + CC * t + j + 16 * k2];
                }
            }
        }
        // inverse DFT along x of each row
        float2* row = buf + g * P;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
#pragma unroll
            for (int j = 0; j < CC; ++j) {
                const int k1 = CC * t + j;
                float2 u[R2];
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) u[k2] = w[i][j * R2 + k2];
                RegDFT<R2, true, float>::run(u);
#pragma unroll
                for (int tt = 1; tt < R2; ++tt) u[tt] = mulc<float>(u[tt], tw_i[tt * 16 + k1]);
#pragma unroll
                for (int tt = 0; tt < R2; ++tt) w[i][j * R2 + tt] = u[tt];
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < CC; ++j)
#pragma unroll
                for (int tt = 0; tt < R2; ++tt) row[xpos<R2>(CC * t + j, tt)] = w[i][j * R2 + tt];
            __syncthreads();
#pragma unroll
            for (int k1 = 0; k1 < 16; ++k1) w[i][k1] = row[xpos<R2>(k1, t)];
            dft16<float, true>(w[i]);
        }
        // the imaginary part of a lone last field (rounding only) goes back to its
        // workspace plane, which this block has finished reading
        float* __restrict__ out0 = a.out + (long long)(2 * pair) * a.n + (long long)y * NX;
        float* __restrict__ out1 = has_b ? out0 + a.n : a.lone + (long long)y * NX;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int off = (g + G * i) * pl + t + R2 * r;
                __builtin_nontemporal_store(w[i][r].x, out0 + off);
                __builtin_nontemporal_store(w[i][r].y, out1 + off);
            }
        }
    }
}

// y pass: W = 16 adjacent x frequencies (columns of the re and im planes) x NY points
// at one theta frequency, for one pair of the batch (the backward: every pair in turn).
// Columns per workgroup: 32 (128-byte row segments per plane, one workgroup round at
// 256^2 x 64) where the LDS allows; the backward keeps 16 (its accumulator and table
// registers limit occupancy either way).
template <int NY, int MODE> struct YFullW {
    static constexpr int W = ((MODE <= 1 || MODE == 4) && NY <= 256) ? 32 : 16;
};

template <int NY, int MODE> struct FullLineGeom {
    static constexpr int R1 = NY > 256 ? 32 : 16;
    static constexpr int R2 = NY / R1;
    static constexpr int CC = R1 / R2;
    static constexpr int W = YFullW<NY, MODE>::W;
    static constexpr int NT = W * R2;
};

template <int NY, int MODE>
static constexpr size_t full_line_lds() {
    return sizeof(float2) * ((size_t)NY * FullLineGeom<NY, MODE>::W + 2 * NY);
}

// scale * prod_e T_e at (kt, ky, kx), conjugated for the adjoint
__device__ __forceinline__ float2 full_table_factor(const FullFastArgs& a, int NYv, int kt, int ky, int kx,
                                                    float scale) {
    const int pl = a.nx * NYv;
    float2 f = make_float2(scale, 0.f);
    for (int e = 0; e < a.ntab; ++e) {
        const float2* T = reinterpret_cast<const float2*>(a.tab[e]);
        if (a.tab_full[e] == 1) {
            f = mul<float>(f, T[(long long)kt * pl + ky * a.nx + kx]);
        } else if (a.tab_full[e] == 2) {
            f = mul<float>(f, T[quarter_offset(kt, ky, kx, a.nx, NYv)]);
        } else {
            f = mul<float>(f, T[kx]);
            f = mul<float>(f, T[a.nx + ky]);
            f = mul<float>(f, T[a.nx + NYv + kt]);
        }
    }
    if (a.conj_tab) f.y = -f.y;
    return f;
}

// MODE 0 (convolve): forward DFT along y, [copy of the spectrum to save], product
//   with scale * prod T (conjugated for the adjoint), inverse DFT, in place.
// MODE 1 (spectra): forward DFT along y written to save; nothing else.
// MODE 2 (backward): as MODE 0 on the upstream gradient g (the adjoint product), and
//   in the same sweep A[k] = sum_pairs Z_g[k] conj(Z_f[k]) with the field spectra Z_f
//   (zf); at the end W[k] A[k] / n^2 goes through the inverse DFT along y to acc (two
//   planes).  Its x-theta inverse has real part dL/dP summed over the batch.
// TK: the chain is one FULL table (1) or one quarter table (2), read with 32-bit offsets
// (the general product loop, compiled in, would cost the registers of a fourth wave per
// SIMD); 0: any chain.
template <int NY, int MODE, int TK = 0>
__global__ void __launch_bounds__((FullLineGeom<NY, MODE>::NT)) y_full(FullFastArgs a) {
    using Gm = FullLineGeom<NY, MODE>;
    constexpr int R1 = Gm::R1, R2 = Gm::R2, CC = Gm::CC, W = Gm::W, NT = Gm::NT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* buf = reinterpret_cast<float2*>(smem_raw);  // [k1*R2 + t][W]
    float2* tw_f = buf + NY * W;                        // [k1][t] = w_NY^{t k1}
    float2* tw_i = tw_f + NY;                           // [t][k1]
    const int tid = threadIdx.x;
    for (int i = tid; i < NY; i += NT) {
        const int k1 = i / R2, t = i - k1 * R2;
        const float2 w = a.twy[t * k1];
        tw_f[k1 * R2 + t] = w;
        tw_i[t * R1 + k1] = w;
    }
    __syncthreads();

    const int ctiles = a.nx / W;
    const int pl = a.nx * NY;
    const int npairs = (a.batch + 1) / 2;
    // MODE 0 and 1: one pair per workgroup, the workgroups of one column tile (its pairs)
    // back to back on one XCD, so that the tile's table entries come from HBM once and are
    // then L2 hits (the backward's accumulator needs every pair in one workgroup)
    const int bid = xcd_contiguous(blockIdx.x, gridDim.x);
    const int tb = MODE == 2 ? bid : bid / npairs;
    const int p_lo = MODE == 2 ? 0 : bid - tb * npairs;
    const int p_hi = MODE == 2 ? npairs : p_lo + 1;
    const int kt = tb / ctiles;
    const int ct = tb - kt * ctiles;
    // table factor for (kt, ky = k1 + R1 k2, kx), k1 = CC t + j: held in registers across
    // the pair loop by the backward; the convolution reads it once per workgroup, in the
    // product, which keeps it within 128 registers (four waves per SIMD)
    float2 tv[CC][R2];
    if constexpr (MODE == 2) {
        const int q = tid % W, t = tid / W;
        const int kx = ct * W + q;
#pragma unroll
        for (int j = 0; j < CC; ++j)
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2)
                tv[j][k2] = full_table_factor(a, NY, kt, CC * t + j + R1 * k2, kx, a.scale);
    }
    float2 acc[CC][R2];
    if constexpr (MODE == 2) {
#pragma unroll
        for (int j = 0; j < CC; ++j)
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) acc[j][k2] = make_float2(0.f, 0.f);
    }
    const int rstride = R2 * a.nx;
    for (int pair = p_lo; pair < p_hi; ++pair) {
        // per-lane offsets are recomputed for every pair rather than hoisted out of the
        // loop (hoisting them would hold dozens of registers across the loop)
        int lt = tid;
        asm volatile("" : "+v"(lt));
        const int q = lt % W, t = lt / W;
        const int base = kt * pl + ct * W + q;  // element (kt, y, kx) at base + y nx
        const int lane_off = base + t * a.nx;
        float* __restrict__ re = a.out + (long long)(2 * pair) * a.n;
        float* __restrict__ im = 2 * pair + 1 < a.batch ? re + a.n : a.lone;
        float2 w[R1];
        float2 u[CC][R2];
        if constexpr (MODE == 4) {
            // the y spectrum at ky = CC t + j + R1 k2, as the forward pass leaves it
#pragma unroll
            for (int j = 0; j < CC; ++j)
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) {
                    const int off = base + (CC * t + j + R1 * k2) * a.nx;
                    u[j][k2] = make_float2(re[off], im[off]);
                }
        } else {
#pragma unroll
            for (int r = 0; r < R1; ++r) w[r] = make_float2(re[lane_off + r * rstride], im[lane_off + r * rstride]);
            RegDFT<R1, false, float>::run(w);
#pragma unroll
            for (int k1 = 1; k1 < R1; ++k1) w[k1] = mul<float>(w[k1], tw_f[k1 * R2 + t]);
            __syncthreads();
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) buf[(k1 * R2 + t) * W + q] = w[k1];
            __syncthreads();
#pragma unroll
            for (int j = 0; j < CC; ++j) {
                const int k1 = CC * t + j;
#pragma unroll
                for (int tt = 0; tt < R2; ++tt) u[j][tt] = buf[(k1 * R2 + tt) * W + q];
                RegDFT<R2, false, float>::run(u[j]);
            }
        }
        if (MODE == 1 || (MODE != 4 && a.save)) {
            float* s_re = a.save + (long long)(2 * pair) * a.n;
            float* s_im = (2 * pair + 1 < a.batch || !a.save_lone) ? s_re + a.n : a.save_lone;
#pragma unroll
            for (int j = 0; j < CC; ++j)
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) {
                    const int off = base + (CC * t + j + R1 * k2) * a.nx;
                    s_re[off] = u[j][k2].x;
                    s_im[off] = u[j][k2].y;
                }
        }
        if constexpr (MODE == 1) continue;
        if constexpr (MODE == 2) {
            const float* z_re = a.zf + (long long)(2 * pair) * a.n;
            const float* z_im = z_re + a.n;
#pragma unroll
            for (int j = 0; j < CC; ++j)
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) {
                    const int off = base + (CC * t + j + R1 * k2) * a.nx;
                    const float2 z = make_float2(z_re[off], z_im[off]);
                    acc[j][k2].x += u[j][k2].x * z.x + u[j][k2].y * z.y;  // u conj(z)
                    acc[j][k2].y += u[j][k2].y * z.x - u[j][k2].x * z.y;
                }
        }
#pragma unroll
        for (int j = 0; j < CC; ++j) {
            const int k1 = CC * t + j;
            if constexpr (MODE == 4) {
                // inverse only: no product
            } else if constexpr (MODE == 2) {
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) u[j][k2] = mul<float>(u[j][k2], tv[j][k2]);
            } else if constexpr (TK == 1) {
                // one FULL table: 32-bit byte offsets from the uniform table base
                const char* T = reinterpret_cast<const char*>(a.tab[0]);
                const unsigned o0 = (unsigned)(base + k1 * a.nx) * 8u;
                const unsigned ostep = (unsigned)(R1 * a.nx) * 8u;
                const float sc = a.scale, sg = a.conj_tab ? -a.scale : a.scale;
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) {
                    const float2 tf = *reinterpret_cast<const float2*>(T + (o0 + (unsigned)k2 * ostep));
                    u[j][k2] = mul<float>(u[j][k2], make_float2(tf.x * sc, tf.y * sg));
                }
            } else if constexpr (TK == 2) {
                // one quarter table: row |ky| of plane kt, column |kx|
                const float2* T = reinterpret_cast<const float2*>(a.tab[0]);
                const int kx = ct * W + q;
                const int hx = a.nx / 2 + 1;
                const int col = min(kx, a.nx - kx);
                const int row0 = kt * (NY / 2 + 1);
                const float sc = a.scale, sg = a.conj_tab ? -a.scale : a.scale;
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) {
                    const int ky = k1 + R1 * k2;
                    const float2 tf = T[(row0 + min(ky, NY - ky)) * hx + col];
                    u[j][k2] = mul<float>(u[j][k2], make_float2(tf.x * sc, tf.y * sg));
                }
            } else {
                const int kx = base - kt * pl;
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2)
                    u[j][k2] = mul<float>(u[j][k2], full_table_factor(a, NY, kt, k1 + R1 * k2, kx, a.scale));
            }
            RegDFT<R2, true, float>::run(u[j]);
#pragma unroll
            for (int tt = 1; tt < R2; ++tt) u[j][tt] = mulc<float>(u[j][tt], tw_i[tt * R1 + k1]);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CC; ++j)
#pragma unroll
            for (int tt = 0; tt < R2; ++tt) buf[((CC * t + j) * R2 + tt) * W + q] = u[j][tt];
        __syncthreads();
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) w[k1] = buf[(k1 * R2 + t) * W + q];
        RegDFT<R1, true, float>::run(w);
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            re[lane_off + r * rstride] = w[r].x;
            im[lane_off + r * rstride] = w[r].y;
        }
    }
    if constexpr (MODE == 2) {
        // W[k] = (-1)^(kx + ky) and 1/n^2, then the inverse DFT along y of the accumulator
        const int q = tid % W, t = tid / W;
        const int kx = ct * W + q;
        const int base = kt * pl + kx;
        const float s2 = a.acc_scale;
#pragma unroll
        for (int j = 0; j < CC; ++j) {
            const int k1 = CC * t + j;
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) {
                const int ky = k1 + R1 * k2;
                const float sg = ((kx + ky) & 1) ? -s2 : s2;
                acc[j][k2] = make_float2(acc[j][k2].x * sg, acc[j][k2].y * sg);
            }
            RegDFT<R2, true, float>::run(acc[j]);
#pragma unroll
            for (int tt = 1; tt < R2; ++tt) acc[j][tt] = mulc<float>(acc[j][tt], tw_i[tt * R1 + k1]);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CC; ++j)
#pragma unroll
            for (int tt = 0; tt < R2; ++tt) buf[((CC * t + j) * R2 + tt) * W + q] = acc[j][tt];
        __syncthreads();
        float2 w[R1];
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) w[k1] = buf[(k1 * R2 + t) * W + q];
        RegDFT<R1, true, float>::run(w);
        float* __restrict__ o_re = a.acc;
        float* __restrict__ o_im = a.acc + a.n;
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            const int off = base + (t + R2 * r) * a.nx;
            o_re[off] = w[r].x;
            o_im[off] = w[r].y;
        }
    }
}

// ------------------------------------------------------------------ dispatch
bool full_fast_supported(int nx, int ny, int m) {
    return (nx == 32 || nx == 64 || nx == 128 || nx == 256) && (m == 16 || m == 32 || m == 64) &&
           (ny == 32 || ny == 64 || ny == 128 || ny == 256 || ny == 512);
}

template <int NX, int M, int DIR>
static hipError_t launch_xt_full_t(const FullFastArgs& a, hipStream_t s) {
    const int nblocks = ((a.batch + 1) / 2) * a.ny;
    const int nthr = FullSlabGeom<NX, M>::NT;
    const size_t lds = full_slab_lds<NX, M>();
    hipLaunchKernelGGL((xt_full<NX, M, DIR>), dim3(nblocks), dim3(nthr), lds, s, a);
    return hipGetLastError();
}

#define SE2C_XT_FULL_CASE(NX_, M_) \
    if (a.nx == NX_ && a.m == M_) return launch_xt_full_t<NX_, M_, DIR>(a, s);

template <int DIR>
static hipError_t launch_xt_full(const FullFastArgs& a, hipStream_t s) {
    SE2C_XT_FULL_CASE(32, 16) SE2C_XT_FULL_CASE(32, 32) SE2C_XT_FULL_CASE(32, 64)
    SE2C_XT_FULL_CASE(64, 16) SE2C_XT_FULL_CASE(64, 32) SE2C_XT_FULL_CASE(64, 64)
    SE2C_XT_FULL_CASE(128, 16) SE2C_XT_FULL_CASE(128, 32) SE2C_XT_FULL_CASE(128, 64)
    SE2C_XT_FULL_CASE(256, 16) SE2C_XT_FULL_CASE(256, 32) SE2C_XT_FULL_CASE(256, 64)
    return hipErrorInvalidValue;
}

hipError_t launch_xt_full_fwd(const FullFastArgs& a, hipStream_t s) { return launch_xt_full<0>(a, s); }
hipError_t launch_xt_full_inv(const FullFastArgs& a, hipStream_t s) { return launch_xt_full<1>(a, s); }
hipError_t launch_x_full_fwd(const FullFastArgs& a, hipStream_t s) { return launch_xt_full<2>(a, s); }

// All powers (Alg. 7) along y, MODE 3 geometry: each workgroup (theta frequency, 16 x
// frequencies) walks the pairs; a pair's y spectrum Z (forward DFT of the x-theta spectrum
// planes in the last output slot) stays in registers while, for p = 1..q, the running
// product H_p = H_{p-1} T (H_0 = Z / n, conjugated for the adjoint) is inverted along y
// into slot p - 1.  The last slot is read before it is written (same workgroup, same
// pair).  Up to NY = 256 the workgroup's table tile (NY x 16 factors, the chain's product)
// sits in LDS, read from HBM once for all pairs and powers; at NY = 512 it would leave one
// workgroup per CU, and the factor is read from memory for every power.
template <int NY> struct PowersGeom {
    static constexpr bool TAB_LDS = NY <= 256;
};
template <int NY>
static constexpr size_t powers_lds() {
    return full_line_lds<NY, 3>() +
           (PowersGeom<NY>::TAB_LDS ? sizeof(float2) * (size_t)NY * FullLineGeom<NY, 3>::W : 0);
}

template <int NY>
__global__ void __launch_bounds__((FullLineGeom<NY, 3>::NT)) y_full_powers(FullFastArgs a) {
    using Gm = FullLineGeom<NY, 3>;
    constexpr int R1 = Gm::R1, R2 = Gm::R2, CC = Gm::CC, W = Gm::W, NT = Gm::NT;
    constexpr bool TL = PowersGeom<NY>::TAB_LDS;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* buf = reinterpret_cast<float2*>(smem_raw);  // [k1*R2 + t][W]
    float2* tw_f = buf + NY * W;                        // [k1][t] = w_NY^{t k1}
    float2* tw_i = tw_f + NY;                           // [t][k1]
    float2* tabl = tw_i + NY;                           // [ky][W] (TL)
    const int tid = threadIdx.x;
    for (int i = tid; i < NY; i += NT) {
        const int k1 = i / R2, t = i - k1 * R2;
        const float2 w = a.twy[t * k1];
        tw_f[k1 * R2 + t] = w;
        tw_i[t * R1 + k1] = w;
    }
    const int ctiles = a.nx / W;
    const int bid = xcd_contiguous(blockIdx.x, gridDim.x);
    const int kt = bid / ctiles;
    const int ct = bid - kt * ctiles;
    if constexpr (TL) {
        for (int i = tid; i < NY * W; i += NT) {
            const int ky = i / W;
            tabl[i] = full_table_factor(a, NY, kt, ky, ct * W + (i - ky * W), 1.0f);
        }
    }
    __syncthreads();

    const int pl = a.nx * NY;
    const int npairs = a.batch / 2;
    const int rstride = R2 * a.nx;
    const float* __restrict__ spec = a.out + (long long)(a.q - 1) * a.slot;
    for (int pair = 0; pair < npairs; ++pair) {
        int lt = tid;
        asm volatile("" : "+v"(lt));
        const int q = lt % W, t = lt / W;
        const int base = kt * pl + ct * W + q;
        const int lane_off = base + t * a.nx;
        const float* __restrict__ sre = spec + (long long)(2 * pair) * a.n;
        const float* __restrict__ sim = sre + a.n;
        float2 w[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r) w[r] = make_float2(sre[lane_off + r * rstride], sim[lane_off + r * rstride]);
        RegDFT<R1, false, float>::run(w);
#pragma unroll
        for (int k1 = 1; k1 < R1; ++k1) w[k1] = mul<float>(w[k1], tw_f[k1 * R2 + t]);
        __syncthreads();
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) buf[(k1 * R2 + t) * W + q] = w[k1];
        __syncthreads();
        float2 h[CC][R2];  // running product H_p
#pragma unroll
        for (int j = 0; j < CC; ++j) {
            const int k1 = CC * t + j;
#pragma unroll
            for (int tt = 0; tt < R2; ++tt) h[j][tt] = buf[(k1 * R2 + tt) * W + q];
            RegDFT<R2, false, float>::run(h[j]);
#pragma unroll
            for (int tt = 0; tt < R2; ++tt) h[j][tt] = make_float2(h[j][tt].x * a.scale, h[j][tt].y * a.scale);
        }
#pragma unroll 1
        for (int pw = 0; pw < a.q; ++pw) {
            float2 u[CC][R2];
#pragma unroll
            for (int j = 0; j < CC; ++j) {
                const int k1 = CC * t + j;
                const int kx = base - kt * pl;
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) {
                    const float2 tf = TL ? tabl[(k1 + R1 * k2) * W + q]
                                         : full_table_factor(a, NY, kt, k1 + R1 * k2, kx, 1.0f);
                    h[j][k2] = mul<float>(h[j][k2], tf);
                }
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) u[j][k2] = h[j][k2];
                RegDFT<R2, true, float>::run(u[j]);
#pragma unroll
                for (int tt = 1; tt < R2; ++tt) u[j][tt] = mulc<float>(u[j][tt], tw_i[tt * R1 + k1]);
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < CC; ++j)
#pragma unroll
                for (int tt = 0; tt < R2; ++tt) buf[((CC * t + j) * R2 + tt) * W + q] = u[j][tt];
            __syncthreads();
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) w[k1] = buf[(k1 * R2 + t) * W + q];
            RegDFT<R1, true, float>::run(w);
            float* __restrict__ ore = a.out + (long long)pw * a.slot + (long long)(2 * pair) * a.n;
            float* __restrict__ oim = ore + a.n;
#pragma unroll
            for (int r = 0; r < R1; ++r) {
                ore[lane_off + r * rstride] = w[r].x;
                oim[lane_off + r * rstride] = w[r].y;
            }
        }
    }
}

// prod_e T_e at (kt, ky, kx) of a grid lx x ly (tables of the sampling grid), conjugated
// for the adjoint (no scale)
__device__ __forceinline__ float2 grid_table_factor(const FullFastArgs& a, int lx, int ly, int kt, int ky, int kx) {
    float2 f = make_float2(1.f, 0.f);
    for (int e = 0; e < a.ntab; ++e) {
        const float2* T = reinterpret_cast<const float2*>(a.tab[e]);
        if (a.tab_full[e] == 1) {
            f = mul<float>(f, T[((long long)kt * ly + ky) * lx + kx]);
        } else if (a.tab_full[e] == 2) {
            f = mul<float>(f, T[quarter_offset(kt, ky, kx, lx, ly)]);
        } else {
            f = mul<float>(f, T[kx]);
            f = mul<float>(f, T[lx + ky]);
            f = mul<float>(f, T[lx + ly + kt]);
        }
    }
    if (a.conj_tab) f.y = -f.y;
    return f;
}

// Evaluation on a finer grid (Sec. 4.1 eq. (MatSKfonG)), y pass on the evaluation grid
// (NY its Ny), MODE 3 geometry: each workgroup (theta frequency, 16 x frequencies of the
// evaluation grid) walks the pairs.  A lane's values come from the sampling-grid y spectra
// (zsrc, two planes per pair) at the padded indices of each axis (pad_source: the same
// signed frequency; an even length's Nyquist index halved when the grid is finer), times
// the sampling-grid table factor and scale; zero for frequencies the sampling grid lacks.
// Then the inverse DFT along y into the evaluation grid's planes (out, two per pair).
template <int NY>
__global__ void __launch_bounds__((FullLineGeom<NY, 3>::NT)) y_full_pad_inv(FullFastArgs a) {
    using Gm = FullLineGeom<NY, 3>;
    constexpr int R1 = Gm::R1, R2 = Gm::R2, CC = Gm::CC, W = Gm::W, NT = Gm::NT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* buf = reinterpret_cast<float2*>(smem_raw);  // [k1*R2 + t][W]
    float2* tw_i = buf + NY * W + NY;                   // [t][k1]
    const int tid = threadIdx.x;
    for (int i = tid; i < NY; i += NT) {
        const int k1 = i / R2, t = i - k1 * R2;
        tw_i[t * R1 + k1] = a.twy[t * k1];
    }
    __syncthreads();

    const int ctiles = a.nx / W;
    const int bid = xcd_contiguous(blockIdx.x, gridDim.x);
    const int kt = bid / ctiles;
    const int ct = bid - kt * ctiles;
    const int pl = a.nx * NY;
    const int npairs = a.batch / 2;
    const int rstride = R2 * a.nx;
    bool ht;
    const int st = pad_source(kt, a.m, a.lm, &ht);
    for (int pair = 0; pair < npairs; ++pair) {
        int lt = tid;
        asm volatile("" : "+v"(lt));
        const int q = lt % W, t = lt / W;
        const int kx = ct * W + q;
        const int lane_off = kt * pl + kx + t * a.nx;
        bool hx;
        const int sx = pad_source(kx, a.nx, a.lx, &hx);
        const float* __restrict__ zre = a.zsrc + (long long)(2 * pair) * a.nl;
        const float* __restrict__ zim = zre + a.nl;
        float wgt = a.scale;
        if (hx) wgt *= 0.5f;
        if (ht) wgt *= 0.5f;
        float2 u[CC][R2];
#pragma unroll
        for (int j = 0; j < CC; ++j) {
            const int k1 = CC * t + j;
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) {
                bool hy;
                const int sy = pad_source(k1 + R1 * k2, NY, a.ly, &hy);
                float2 v = make_float2(0.f, 0.f);
                if (st >= 0 && sx >= 0 && sy >= 0) {
                    const long long o = ((long long)st * a.ly + sy) * a.lx + sx;
                    const float2 f = grid_table_factor(a, a.lx, a.ly, st, sy, sx);
                    const float c = hy ? 0.5f * wgt : wgt;
                    v = mul<float>(make_float2(zre[o] * c, zim[o] * c), f);
                }
                u[j][k2] = v;
            }
            RegDFT<R2, true, float>::run(u[j]);
#pragma unroll
            for (int tt = 1; tt < R2; ++tt) u[j][tt] = mulc<float>(u[j][tt], tw_i[tt * R1 + k1]);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CC; ++j)
#pragma unroll
            for (int tt = 0; tt < R2; ++tt) buf[((CC * t + j) * R2 + tt) * W + q] = u[j][tt];
        __syncthreads();
        float2 w[R1];
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) w[k1] = buf[(k1 * R2 + t) * W + q];
        RegDFT<R1, true, float>::run(w);
        float* __restrict__ ore = a.out + (long long)(2 * pair) * a.n;
        float* __restrict__ oim = ore + a.n;
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            ore[lane_off + r * rstride] = w[r].x;
            oim[lane_off + r * rstride] = w[r].y;
        }
    }
}

// Shift-mix theta pass of a sum of SE(2)-shifted kernels, on the x-y spectrum planes with
// theta still in space: one block per (y frequency ky, 16 x frequencies), PG groups of
// threads taking PG pairs of the batch at a time (every pair of a batch of 8 at once at
// M = 64); the block's shift-phase tiles Q_j[alpha][ky][kx0 .. kx0 + 15] are loaded into
// LDS with the first pairs' tiles and serve every pair.  Per pair:
// z'[alpha] = sum_j z[alpha - r_j] Q_j[alpha - r_j] (indices mod M) from the pair's tile in
// LDS, the forward DFT along theta in registers (M = R1 x R2, one LDS exchange in the same
// tile), the product with the chain's factor at (kx, ky, kt) (scale 1/n, conjugated for the
// adjoint), stored in place; the x-theta inverse pass follows.  Blocks of neighbouring
// column tiles run back to back on one XCD (64-byte rows: halves of the same cache lines).
template <int M> struct ShiftGeom {
    static constexpr int R1 = M == 16 ? 8 : 16;
    static constexpr int R2 = M / R1;
    static constexpr int CC = R1 / R2;
    static constexpr int W = 16;
    static constexpr int LT = W * R2;  // threads per pair group
    static constexpr int PG = 256 / LT;
    static constexpr int NT = LT * PG;
    static_assert(R1 * R2 == M && CC * R2 == R1 && NT == 256, "shift pass geometry");
};

template <int M>
static size_t t_shift_lds(int nshift) {
    using Gm = ShiftGeom<M>;
    return sizeof(float2) * ((size_t)3 * M + (size_t)(nshift + Gm::PG) * M * Gm::W);
}

template <int M>
__global__ void __launch_bounds__(256) t_shift_full(FullFastArgs a) {
    using Gm = ShiftGeom<M>;
    constexpr int R1 = Gm::R1, R2 = Gm::R2, CC = Gm::CC, W = Gm::W, LT = Gm::LT, PG = Gm::PG, NT = Gm::NT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* tw_f = reinterpret_cast<float2*>(smem_raw);  // [k1][t] = w_M^{t k1}
    float2* tw_i = tw_f + M;                             // [t][k1]
    float2* qt = tw_i + M;                               // [j][alpha][W]
    float2* tiles = qt + (size_t)a.nshift * M * W;       // PG x [alpha][W], then the exchange
    float2* ftt = tiles + (size_t)PG * M * W;            // separable chains: scale prod_e Tt_e[kt]
    const int tid = threadIdx.x;
    for (int i = tid; i < M; i += NT) {
        const int k1 = i / R2, t = i - k1 * R2;
        const float2 w = a.twt[t * k1];
        tw_f[k1 * R2 + t] = w;
        tw_i[t * R1 + k1] = w;
    }
    bool sep = true;
    for (int e = 0; e < a.ntab; ++e) sep = sep && a.tab_full[e] == 0;
    if (sep)
        for (int i = tid; i < M; i += NT) {
            float2 f = make_float2(a.scale, 0.f);
            for (int e = 0; e < a.ntab; ++e)
                f = mul<float>(f, reinterpret_cast<const float2*>(a.tab[e])[a.nx + a.ny + i]);
            if (a.conj_tab) f.y = -f.y;
            ftt[i] = f;
        }
    const int ctiles = a.nx / W;
    const int bid = xcd_contiguous(blockIdx.x, gridDim.x);
    const int ky = bid / ctiles;
    const int kx0 = (bid - ky * ctiles) * W;
    const long long plane = (long long)a.nx * a.ny;
    const long long col0 = (long long)ky * a.nx + kx0;
    for (int i = tid; i < a.nshift * M * W; i += NT) {
        const int j = i / (M * W);
        const int rem = i - j * (M * W);
        const int al = rem / W;
        qt[i] = a.qtab[(long long)j * a.n + al * plane + col0 + (rem - al * W)];
    }

    const int g = tid / LT, lt = tid - g * LT;
    const int q = lt % W, t = lt / W;
    float2* tile = tiles + (size_t)g * M * W;
    const int npairs = (a.batch + 1) / 2;
    for (int p0 = 0; p0 < npairs; p0 += PG) {
        const int pair = p0 + g;
        const bool active = pair < npairs;
        float* __restrict__ re = a.out + (long long)(2 * pair) * a.n;
        float* __restrict__ im = 2 * pair + 1 < a.batch ? re + a.n : a.lone;
        if (p0 > 0) __syncthreads();  // the previous pairs' exchange reads are done
        if (active) {
#pragma unroll
            for (int r = 0; r < R1; ++r) {
                const int al = t + R2 * r;
                const long long off = al * plane + col0 + q;
                tile[al * W + q] = make_float2(re[off], im[off]);
            }
        }
        __syncthreads();  // tiles (and, the first time, the twiddles and Q tiles) in LDS
        float2 w[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            const int al = t + R2 * r;
            float2 acc = make_float2(0.f, 0.f);
            for (int j = 0; j < a.nshift; ++j) {
                int src = al - a.rolls[j];
                if (src < 0) src += M;
                const float2 z = tile[src * W + q];
                const float2 f = qt[(j * M + src) * W + q];
                acc.x = fmaf(z.x, f.x, fmaf(-z.y, f.y, acc.x));
                acc.y = fmaf(z.x, f.y, fmaf(z.y, f.x, acc.y));
            }
            w[r] = acc;
        }
        RegDFT<R1, false, float>::run(w);
#pragma unroll
        for (int k1 = 1; k1 < R1; ++k1) w[k1] = mul<float>(w[k1], tw_f[k1 * R2 + t]);
        __syncthreads();  // every mix read of the tiles is done: they become the exchange buffers
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) tile[(k1 * R2 + t) * W + q] = w[k1];
        __syncthreads();
        if (active) {
            const int kx = kx0 + q;
            // separable chains: the x-y part of the factor once, the theta part from LDS
            float2 fxy = make_float2(1.f, 0.f);
            if (sep) {
                for (int e = 0; e < a.ntab; ++e) {
                    const float2* T = reinterpret_cast<const float2*>(a.tab[e]);
                    fxy = mul<float>(fxy, mul<float>(T[kx], T[a.nx + ky]));
                }
                if (a.conj_tab) fxy.y = -fxy.y;
            }
            // one first-stage frequency at a time (the chain's factor loop, unrolled over
            // every value, would hold its loads in a few hundred registers)
#pragma unroll 1
            for (int j = 0; j < CC; ++j) {
                const int k1 = CC * t + j;
                float2 u[R2];
#pragma unroll
                for (int tt = 0; tt < R2; ++tt) u[tt] = tile[(k1 * R2 + tt) * W + q];
                RegDFT<R2, false, float>::run(u);
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) {
                    const int kt = k1 + R1 * k2;
                    const float2 fac = sep ? mul<float>(fxy, ftt[kt]) : full_table_factor(a, a.ny, kt, ky, kx, a.scale);
                    const float2 v = mul<float>(u[k2], fac);
                    const long long off = kt * plane + col0 + q;
                    re[off] = v.x;
                    im[off] = v.y;
                }
            }
        }
    }
}

bool t_shift_supported(int nx, int m, int nshift) {
    if (nx % ShiftGeom<16>::W != 0 || nshift < 1 || nshift > SE2C_MAX_SHIFT_CLASSES) return false;
    size_t lds = 0;
    if (m == 16) lds = t_shift_lds<16>(nshift);
    else if (m == 32) lds = t_shift_lds<32>(nshift);
    else if (m == 64) lds = t_shift_lds<64>(nshift);
    else return false;
    return lds <= 128 * 1024;
}

template <int M>
static hipError_t launch_t_shift_t(const FullFastArgs& a, hipStream_t s) {
    const int nblocks = a.ny * (a.nx / ShiftGeom<M>::W);
    hipLaunchKernelGGL((t_shift_full<M>), dim3(nblocks), dim3(256), t_shift_lds<M>(a.nshift), s, a);
    return hipGetLastError();
}

hipError_t launch_t_shift(const FullFastArgs& a, hipStream_t s) {
    if (!t_shift_supported(a.nx, a.m, a.nshift)) return hipErrorInvalidValue;
    if (a.m == 16) return launch_t_shift_t<16>(a, s);
    if (a.m == 32) return launch_t_shift_t<32>(a, s);
    return launch_t_shift_t<64>(a, s);
}

template <int NY, int MODE>
static hipError_t launch_y_full_t(const FullFastArgs& a, hipStream_t s) {
    const int nblocks = (a.nx / FullLineGeom<NY, MODE>::W) * a.m * (MODE == 2 ? 1 : (a.batch + 1) / 2);
    const int nthr = FullLineGeom<NY, MODE>::NT;
    const size_t lds = full_line_lds<NY, MODE>();
    if (MODE == 0 && a.ntab == 1 && a.tab_full[0] == 1)
        hipLaunchKernelGGL((y_full<NY, MODE, 1>), dim3(nblocks), dim3(nthr), lds, s, a);
    else if (MODE == 0 && a.ntab == 1 && a.tab_full[0] == 2)
        hipLaunchKernelGGL((y_full<NY, MODE, 2>), dim3(nblocks), dim3(nthr), lds, s, a);
    else
        hipLaunchKernelGGL((y_full<NY, MODE, 0>), dim3(nblocks), dim3(nthr), lds, s, a);
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_y_full_mode(const FullFastArgs& a, hipStream_t s) {
    if (a.ny == 32) return launch_y_full_t<32, MODE>(a, s);
    if (a.ny == 64) return launch_y_full_t<64, MODE>(a, s);
    if (a.ny == 128) return launch_y_full_t<128, MODE>(a, s);
    if (a.ny == 256) return launch_y_full_t<256, MODE>(a, s);
    if (a.ny == 512) return launch_y_full_t<512, MODE>(a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_y_full(const FullFastArgs& a, hipStream_t s) { return launch_y_full_mode<0>(a, s); }
hipError_t launch_y_full_spectra(const FullFastArgs& a, hipStream_t s) { return launch_y_full_mode<1>(a, s); }
hipError_t launch_y_full_backward(const FullFastArgs& a, hipStream_t s) { return launch_y_full_mode<2>(a, s); }
hipError_t launch_y_full_inverse(const FullFastArgs& a, hipStream_t s) { return launch_y_full_mode<4>(a, s); }

template <int NY>
static hipError_t launch_y_full_powers_t(const FullFastArgs& a, hipStream_t s) {
    const int nblocks = (a.nx / FullLineGeom<NY, 3>::W) * a.m;
    const int nthr = FullLineGeom<NY, 3>::NT;
    const size_t lds = powers_lds<NY>();
    hipLaunchKernelGGL((y_full_powers<NY>), dim3(nblocks), dim3(nthr), lds, s, a);
    return hipGetLastError();
}

template <int NY>
static hipError_t launch_y_full_pad_inv_t(const FullFastArgs& a, hipStream_t s) {
    const int nblocks = (a.nx / FullLineGeom<NY, 3>::W) * a.m;
    const int nthr = FullLineGeom<NY, 3>::NT;
    const size_t lds = full_line_lds<NY, 3>();
    hipLaunchKernelGGL((y_full_pad_inv<NY>), dim3(nblocks), dim3(nthr), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_y_full_pad_inv(const FullFastArgs& a, hipStream_t s) {
    if ((a.batch & 1) || a.lx > a.nx || a.ly > a.ny || a.lm > a.m) return hipErrorInvalidValue;
    if (a.ny == 32) return launch_y_full_pad_inv_t<32>(a, s);
    if (a.ny == 64) return launch_y_full_pad_inv_t<64>(a, s);
    if (a.ny == 128) return launch_y_full_pad_inv_t<128>(a, s);
    if (a.ny == 256) return launch_y_full_pad_inv_t<256>(a, s);
    if (a.ny == 512) return launch_y_full_pad_inv_t<512>(a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_y_full_powers(const FullFastArgs& a, hipStream_t s) {
    if ((a.batch & 1) || a.q < 1) return hipErrorInvalidValue;
    if (a.ny == 32) return launch_y_full_powers_t<32>(a, s);
    if (a.ny == 64) return launch_y_full_powers_t<64>(a, s);
    if (a.ny == 128) return launch_y_full_powers_t<128>(a, s);
    if (a.ny == 256) return launch_y_full_powers_t<256>(a, s);
    if (a.ny == 512) return launch_y_full_powers_t<512>(a, s);
    return hipErrorInvalidValue;
}

#define SE2C_XT_FULL_ATTR(NX_, M_)                                                                          \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(xt_full<NX_, M_, 0>),                              \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)full_slab_lds<NX_, M_>());      \
    if (e != hipSuccess) return e;                                                                          \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(xt_full<NX_, M_, 1>),                              \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)full_slab_lds<NX_, M_>());      \
    if (e != hipSuccess) return e;                                                                          \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(xt_full<NX_, M_, 2>),                              \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)full_slab_lds<NX_, M_>());      \
    if (e != hipSuccess) return e;
#define SE2C_Y_FULL_ATTR1(NY_, MODE_)                                                                       \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(y_full<NY_, MODE_>),                               \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)full_line_lds<NY_, MODE_>());   \
    if (e != hipSuccess) return e;
#define SE2C_Y_FULL_ATTR(NY_)                                                                               \
    SE2C_Y_FULL_ATTR1(NY_, 0) SE2C_Y_FULL_ATTR1(NY_, 1) SE2C_Y_FULL_ATTR1(NY_, 2) SE2C_Y_FULL_ATTR1(NY_, 4)   \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(y_full<NY_, 0, 1>),                                \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)full_line_lds<NY_, 0>());       \
    if (e != hipSuccess) return e;                                                                          \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(y_full<NY_, 0, 2>),                                \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)full_line_lds<NY_, 0>());       \
    if (e != hipSuccess) return e;                                                                          \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(y_full_pad_inv<NY_>),                              \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)full_line_lds<NY_, 3>());       \
    if (e != hipSuccess) return e;                                                                          \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(y_full_powers<NY_>),                               \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)powers_lds<NY_>());             \
    if (e != hipSuccess) return e;

hipError_t prepare_full_fast_kernels() {
    hipError_t e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(t_shift_full<16>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(t_shift_full<32>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(t_shift_full<64>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    if (e != hipSuccess) return e;
    SE2C_XT_FULL_ATTR(32, 16) SE2C_XT_FULL_ATTR(32, 32) SE2C_XT_FULL_ATTR(32, 64)
    SE2C_XT_FULL_ATTR(64, 16) SE2C_XT_FULL_ATTR(64, 32) SE2C_XT_FULL_ATTR(64, 64)
    SE2C_XT_FULL_ATTR(128, 16) SE2C_XT_FULL_ATTR(128, 32) SE2C_XT_FULL_ATTR(128, 64)
    SE2C_XT_FULL_ATTR(256, 16) SE2C_XT_FULL_ATTR(256, 32) SE2C_XT_FULL_ATTR(256, 64)
    SE2C_Y_FULL_ATTR(32) SE2C_Y_FULL_ATTR(64) SE2C_Y_FULL_ATTR(128) SE2C_Y_FULL_ATTR(256) SE2C_Y_FULL_ATTR(512)
    return hipSuccess;
}

}  // namespace se2c
