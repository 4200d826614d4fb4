// Pass kernels of the convolutional finite Fourier series on an Nx x Ny x M grid.
//
// Data layout in HBM: real samples F[item][theta][y][x], x fastest (the memory
// order of the paper's F(i, j, l), Sec. 3.2 eq. (OmL)).
//
// Real fields are complexified two at a time (z = a + i b) so that every
// transform is a full-length complex FFT:
//   * y-pair  : rows y = 2s and 2s+1 of one field (used when y is not transformed
//               in this pass and the kernel table is separable);
//   * x-pair  : columns x = 2c and 2c+1 (a float2 / double2 load);
//   * planes  : two separate real planes, e.g. two fields of a batch, or the
//               real/imaginary planes of an intermediate spectrum.
// Because the convolution kernel is real in space, conv(a + i b) = conv(a) +
// i conv(b), so the pair is separated again just by taking Re and Im.
//
// slab_kernel   : tile = one (theta, x) plane: FFT along x and (optionally)
//                 theta, optional separable spectral product, inverse.
// pencil_kernel : tile = W adjacent columns x one line along y or theta: FFT
//                 along that axis, optional spectral product (1-D factor of a
//                 separable table, or full 3-D table), inverse.
#include "fft_device.hpp"
#include "passes.hpp"
#include "full_fast.hpp"

namespace se2c {

// LDS copy of a plan's tables (tables_slots complex slots; src holds at least the
// bytes they cover, see stage_tw_of on the host).
template <typename T>
__device__ __forceinline__ void load_tables(C<T>* dst, const void* src, const RadixPlan& p, int tid, int nthr) {
    if (!p.rader) {
        const C<T>* s = reinterpret_cast<const C<T>*>(src);
        for (int i = tid; i < p.L; i += nthr) dst[i] = s[i];
        return;
    }
    const int n = p.L - 1;
    const int words = (3 * n * (int)sizeof(C<T>) + 8 * n) / 4;
    const uint32_t* s = reinterpret_cast<const uint32_t*>(src);
    uint32_t* d = reinterpret_cast<uint32_t*>(dst);
    for (int i = tid; i < words; i += nthr) d[i] = s[i];
}

// ---------------------------------------------------------------- slab pass
template <typename T, int MAXV, bool ODD>
__global__ void __launch_bounds__(ODD ? 512 : SE2C_MAX_THREADS(T)) slab_kernel(SlabArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C<T>* tile = reinterpret_cast<C<T>*>(smem_raw);
    const int pitch = a.nx + a.pad;                 // row pitch (complex) in LDS
    const int rows = a.rows_per_tile;
    const int es = a.cplx ? 2 : 1;                  // element stride of the planes (interleaved complex: 2)
    C<T>* twx = tile + rows * pitch;                // plan tables of x, then of theta
    C<T>* twt = twx + tables_slots(a.px, (int)sizeof(C<T>));
    C<T>* fx = twt + tables_slots(a.pt, (int)sizeof(C<T>));  // separable factors (scaled)
    C<T>* ft = fx + a.nx;
    const int tid = threadIdx.x, nthr = blockDim.x;
    // elements per thread staged through registers by tile loads and stores (one in
    // the kernels with odd stages, where staging measured slower)
    constexpr int STG = ODD ? 1 : SE2C_STAGE;

    load_tables<T>(twx, a.twx, a.px, tid, nthr);
    if (a.do_t) load_tables<T>(twt, a.twt, a.pt, tid, nthr);
    if (a.mul) {
        const T sc = (T)a.scale;
        for (int i = tid; i < a.nx; i += nthr) {
            C<T> v = mk<T>(sc, (T)0);
            for (int j = 0; j < a.ntab; ++j) v = mul<T>(v, reinterpret_cast<const C<T>*>(a.tx[j])[i]);
            if (a.conj_tab) v.y = -v.y;
            fx[i] = v;
        }
        if (a.do_t) {
            for (int i = tid; i < a.m; i += nthr) {
                C<T> v = mk<T>((T)1, (T)0);
                for (int j = 0; j < a.ntab; ++j) v = mul<T>(v, reinterpret_cast<const C<T>*>(a.tt[j])[i]);
                if (a.conj_tab) v.y = -v.y;
                ft[i] = v;
            }
        }
    }
    // (twiddles become visible at the first barrier inside the tile loop)

    const long long plane = (long long)a.nx * a.ny;
    const int tiles_per_item = a.nslab * a.ntile_t;
    const int ntiles = tiles_per_item * a.nitems;
    int cur_item = -1;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int item = t / tiles_per_item;
        const int rem = t - item * tiles_per_item;
        const int slab = rem / a.ntile_t;
        const int t0 = (rem - slab * a.ntile_t) * rows;
        const int nrow = min(rows, a.m - t0);  // the last theta chunk may be shorter
        const bool last_odd = (a.lone_in1 != nullptr || a.lone_out1 != nullptr) && item == a.nitems - 1;
        if (a.items && a.mul && item != cur_item) {  // per-item chain factors (uniform branch)
            __syncthreads();
            const SepItem& it = a.items[item];
            const T sc = (T)a.scale;
            for (int i = tid; i < a.nx; i += nthr) {
                C<T> v = mk<T>(sc, (T)0);
                for (int j = 0; j < it.ntab; ++j) v = mul<T>(v, reinterpret_cast<const C<T>*>(it.tab[j])[i]);
                if (a.conj_tab) v.y = -v.y;
                fx[i] = v;
            }
            if (a.do_t) {
                for (int i = tid; i < a.m; i += nthr) {
                    C<T> v = mk<T>((T)1, (T)0);
                    for (int j = 0; j < it.ntab; ++j)
                        v = mul<T>(v, reinterpret_cast<const C<T>*>(it.tab[j])[a.nx + a.ny + i]);
                    if (a.conj_tab) v.y = -v.y;
                    ft[i] = v;
                }
            }
            cur_item = item;
        }

        // ---- load: tile[r][x] for theta = t0 + r
        const T* in0 = a.items ? reinterpret_cast<const T*>(a.items[item].in)
                               : reinterpret_cast<const T*>(a.in0) + (long long)item * a.item_stride_in;
        const T* in1;
        if (a.in_mode == 0) {
            in0 += (long long)(2 * slab) * a.nx;
            in1 = in0 + a.nx;
        } else {
            in0 += (long long)slab * a.nx * es;
            in1 = last_odd ? reinterpret_cast<const T*>(a.lone_in1)
                           : (a.in1 ? reinterpret_cast<const T*>(a.in1) + (long long)item * a.item_stride_in : nullptr);
            if (in1) in1 += (long long)slab * a.nx * es;
        }
        __syncthreads();
        const int P = nrow * a.nx;
        // Tile loads and stores move STG elements per thread at a time, reads first,
        // so that that many HBM reads are in flight together.
#pragma unroll 1
        for (int i0 = tid; i0 < P; i0 += STG * nthr) {
            C<T> v[STG];
#pragma unroll
            for (int k = 0; k < STG; ++k) {
                const int i = i0 + k * nthr;
                if (i < P) {
                    const int r = i / a.nx;
                    const long long off = ((long long)(t0 + r) * plane + (i - r * a.nx)) * es;
                    v[k].x = in0[off];
                    v[k].y = in1 ? in1[off] : (T)0;
                }
            }
#pragma unroll
            for (int k = 0; k < STG; ++k) {
                const int i = i0 + k * nthr;
                if (i < P) {
                    const int r = i / a.nx;
                    tile[r * pitch + (i - r * a.nx)] = v[k];
                }
            }
        }
        __syncthreads();

        // ---- forward
        if (a.fwd) {
            line_fft<T, MAXV, false, ODD>(tile, twx, a.px, 1, pitch, nrow, false, tid, nthr);
            if (a.do_t) line_fft<T, MAXV, false, ODD>(tile, twt, a.pt, pitch, 1, a.nx, true, tid, nthr);
        }
        // ---- separable spectral product: z[kt][kx] *= Tx[kx] * Tt[kt] / (nx*m)
        if (a.mul) {
            for (int i = tid; i < P; i += nthr) {
                const int r = i / a.nx;
                const int x = i - r * a.nx;
                const C<T> f = a.do_t ? mul<T>(fx[x], ft[t0 + r]) : fx[x];
                tile[r * pitch + x] = mul<T>(tile[r * pitch + x], f);
            }
            __syncthreads();
        }
        // ---- inverse
        if (a.inv) {
            if (a.do_t) line_fft<T, MAXV, true, ODD>(tile, twt, a.pt, pitch, 1, a.nx, true, tid, nthr);
            line_fft<T, MAXV, true, ODD>(tile, twx, a.px, 1, pitch, nrow, false, tid, nthr);
        }

        // ---- store
        T* out0 = a.items ? reinterpret_cast<T*>(a.items[item].out)
                          : reinterpret_cast<T*>(a.out0) + (long long)item * a.item_stride_out;
        T* out1;
        if (a.out_mode == 0) {
            out0 += (long long)(2 * slab) * a.nx;
            out1 = out0 + a.nx;
        } else {
            out0 += (long long)slab * a.nx * es;
            out1 = last_odd ? reinterpret_cast<T*>(a.lone_out1)
                            : (a.out1 ? reinterpret_cast<T*>(a.out1) + (long long)item * a.item_stride_out : nullptr);
            if (out1) out1 += (long long)slab * a.nx * es;
        }
#pragma unroll 1
        for (int i0 = tid; i0 < P; i0 += STG * nthr) {
            C<T> v[STG];
#pragma unroll
            for (int k = 0; k < STG; ++k) {
                const int i = i0 + k * nthr;
                if (i < P) {
                    const int r = i / a.nx;
                    v[k] = tile[r * pitch + (i - r * a.nx)];
                }
            }
#pragma unroll
            for (int k = 0; k < STG; ++k) {
                const int i = i0 + k * nthr;
                if (i < P) {
                    const int r = i / a.nx;
                    const long long off = ((long long)(t0 + r) * plane + (i - r * a.nx)) * es;
                    out0[off] = v[k].x;
                    if (out1) out1[off] = v[k].y;
                }
            }
        }
    }
}

// -------------------------------------------------------------- pencil pass
// SHIFT: the instantiation that also carries the shift mix (mul == 3), kept apart so
// that the other pencils keep their register allocation.
template <typename T, int MAXV, bool ODD, bool SHIFT = false>
__global__ void __launch_bounds__((ODD || SHIFT) ? 512 : SE2C_MAX_THREADS(T)) pencil_kernel(PencilArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C<T>* tile = reinterpret_cast<C<T>*>(smem_raw);
    const int L = a.p.L;
    const int pitch = a.W + a.pad;                  // LDS pitch between consecutive axis points
    C<T>* tw = tile + L * pitch;                    // plan tables
    C<T>* f1 = tw + tables_slots(a.p, (int)sizeof(C<T>));
    const int tid = threadIdx.x, nthr = blockDim.x;
    constexpr int STG = ODD ? 1 : SE2C_STAGE;  // as in the slab pass

    load_tables<T>(tw, a.tw, a.p, tid, nthr);
    if (a.mul == 1) {
        const T sc = (T)a.scale;
        for (int i = tid; i < L; i += nthr) {
            C<T> v = mk<T>(sc, (T)0);
            for (int j = 0; j < a.ntab; ++j) v = mul<T>(v, reinterpret_cast<const C<T>*>(a.tab1[j])[i]);
            if (a.conj_tab) v.y = -v.y;
            f1[i] = v;
        }
    }

    const long long plane = (long long)a.nx * a.ny;
    const int es = a.cplx ? 2 : 1;  // element stride of the planes (interleaved complex: 2)
    // element stride along the transform axis (in real elements)
    const long long astride = (a.axis == 1) ? (long long)a.nx : plane;
    const int nother = (a.axis == 1) ? a.m : a.ny;
    const int ncol_tiles = (a.ncols + a.W - 1) / a.W;
    const int tiles_per_item = ncol_tiles * nother;
    const int ntiles = tiles_per_item * a.nitems;
    const int P = L * a.W;
    int cur_item = -1;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        // tiles in XCD order: neighbouring column tiles (halves of the same cache lines)
        // on one XCD back to back, and without per-item tables the items (field pairs) of
        // one tile too, so that a table tile is read from HBM once for all of them.  The
        // shift-mix kernel keeps the plain order (260 against 240 us in XCD order at
        // 256 x 256 x 64, batch 8, two rolls).
        const int u = SHIFT ? t : xcd_contiguous(t, ntiles);
        int item, rem;
        if (a.items || SHIFT) {
            item = u / tiles_per_item;
            rem = u - item * tiles_per_item;
        } else {
            rem = u / a.nitems;
            item = u - rem * a.nitems;
        }
        const int other = rem / ncol_tiles;
        const int c0 = (rem - other * ncol_tiles) * a.W;
        const bool last_odd = (a.lone_in1 != nullptr || a.lone_out1 != nullptr) && item == a.nitems - 1;
        const long long obase = (a.axis == 1) ? (long long)other * plane : (long long)other * a.nx;

        __syncthreads();
        if (a.items && a.mul == 1 && item != cur_item) {  // per-item 1-D factor (uniform branch)
            const SepItem& it = a.items[item];
            const long long off = a.axis == 1 ? a.nx : (long long)a.nx + a.ny;
            const T sc = (T)a.scale;
            for (int i = tid; i < L; i += nthr) {
                C<T> v = mk<T>(sc, (T)0);
                for (int j = 0; j < it.ntab; ++j) v = mul<T>(v, reinterpret_cast<const C<T>*>(it.tab[j])[off + i]);
                if (a.conj_tab) v.y = -v.y;
                f1[i] = v;
            }
            cur_item = item;
            __syncthreads();
        }
        if (a.mode == 0) {
            // x-pair view: complex column c = (x = 2c, x = 2c + 1)
            // with items the pencil runs in place on each field's output (written by the slab pass)
            const T* ibase = a.items ? reinterpret_cast<const T*>(a.items[item].out)
                                     : reinterpret_cast<const T*>(a.in0) + (long long)item * a.item_stride_in;
            const C<T>* in = reinterpret_cast<const C<T>*>(ibase + obase);
#pragma unroll 1
            for (int i0 = tid; i0 < P; i0 += STG * nthr) {
                C<T> v[STG];
#pragma unroll
                for (int k = 0; k < STG; ++k) {
                    const int i = i0 + k * nthr;
                    const int e = i / a.W;
                    const int c = i - e * a.W;
                    v[k] = mk<T>((T)0, (T)0);
                    if (i < P && c0 + c < a.ncols) v[k] = in[(e * astride) / 2 + c0 + c];
                }
#pragma unroll
                for (int k = 0; k < STG; ++k) {
                    const int i = i0 + k * nthr;
                    const int e = i / a.W;
                    if (i < P) tile[e * pitch + (i - e * a.W)] = v[k];
                }
            }
        } else {
            const T* in0 = reinterpret_cast<const T*>(a.in0) + (long long)item * a.item_stride_in + obase * es;
            const T* in1 = last_odd ? reinterpret_cast<const T*>(a.lone_in1)
                                    : (a.in1 ? reinterpret_cast<const T*>(a.in1) + (long long)item * a.item_stride_in : nullptr);
            if (in1) in1 += obase * es;
#pragma unroll 1
            for (int i0 = tid; i0 < P; i0 += STG * nthr) {
                C<T> v[STG];
#pragma unroll
                for (int k = 0; k < STG; ++k) {
                    const int i = i0 + k * nthr;
                    const int e = i / a.W;
                    const int c = i - e * a.W;
                    v[k] = mk<T>((T)0, (T)0);
                    if (i < P && c0 + c < a.ncols) {
                        const long long off = (e * astride + c0 + c) * es;
                        v[k].x = in0[off];
                        v[k].y = in1 ? in1[off] : (T)0;
                    }
                }
#pragma unroll
                for (int k = 0; k < STG; ++k) {
                    const int i = i0 + k * nthr;
                    const int e = i / a.W;
                    if (i < P) tile[e * pitch + (i - e * a.W)] = v[k];
                }
            }
        }
        __syncthreads();

        if (SHIFT && a.mul == 3) {
            // shift mix (theta lines: e = alpha, other = k2, column c0 + c = k1):
            // z'[alpha] = sum_j z[alpha - r_j] Q_j[alpha - r_j][k2][k1], indices mod M
            const C<T>* q = reinterpret_cast<const C<T>*>(a.qtab);
            const long long nn = plane * a.m;
            C<T> g[MAXV];
#pragma unroll
            for (int k = 0; k < MAXV; ++k) {
                const int i = tid + k * nthr;
                g[k] = mk<T>((T)0, (T)0);
                if (i < P) {
                    const int e = i / a.W;
                    const int c = i - e * a.W;
                    if (c0 + c < a.ncols) {
                        for (int j = 0; j < a.nshift; ++j) {
                            int src = e - a.rolls[j];
                            if (src < 0) src += L;
                            const C<T> qv = q[(long long)j * nn + (long long)src * plane + (long long)other * a.nx + c0 + c];
                            g[k] = add<T>(g[k], mul<T>(tile[src * pitch + c], qv));
                        }
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < MAXV; ++k) {
                const int i = tid + k * nthr;
                if (i < P) {
                    const int e = i / a.W;
                    tile[e * pitch + (i - e * a.W)] = g[k];
                }
            }
            __syncthreads();
        }
        if (a.fwd) line_fft<T, MAXV, false, ODD>(tile, tw, a.p, pitch, 1, a.W, true, tid, nthr);
        if (a.mul == 1) {
            for (int i = tid; i < P; i += nthr) {
                const int e = i / a.W;
                const int c = i - e * a.W;
                tile[e * pitch + c] = mul<T>(tile[e * pitch + c], f1[e]);
            }
            __syncthreads();
        } else if (a.mul >= 2) {
            // full-table product: element (kx = c0 + c, ky, kt) with (ky, kt) = (e, other) on
            // y lines and (other, e) on theta lines; a separable table contributes
            // Tx[kx] Ty[ky] Tt[kt].
            const T sc = (T)a.scale;
            for (int i = tid; i < P; i += nthr) {
                const int e = i / a.W;
                const int c = i - e * a.W;
                if (c0 + c < a.ncols) {
                    const int kx = c0 + c;
                    const int ky = a.axis == 1 ? e : other;
                    const int kt = a.axis == 1 ? other : e;
                    C<T> w = mk<T>(sc, (T)0);
                    for (int j = 0; j < a.ntab; ++j) {
                        if (a.tab3[j]) {
                            // FULL [m][ny][nx], or quarter [m][ny/2+1][nx/2+1] at |ky|, |kx|
                            const bool qj = (a.tab3_quarter >> j) & 1u;
                            const int ax = qj ? min(kx, a.nx - kx) : kx;
                            const int ay = qj ? min(ky, a.ny - ky) : ky;
                            const long long off = ((long long)kt * (qj ? a.ny / 2 + 1 : a.ny) + ay) *
                                                      (qj ? a.nx / 2 + 1 : a.nx) + ax;
                            w = mul<T>(w, reinterpret_cast<const C<T>*>(a.tab3[j])[off]);
                        } else {
                            w = mul<T>(w, reinterpret_cast<const C<T>*>(a.sepx[j])[kx]);
                            w = mul<T>(w, reinterpret_cast<const C<T>*>(a.sepy[j])[ky]);
                            w = mul<T>(w, reinterpret_cast<const C<T>*>(a.sept[j])[kt]);
                        }
                    }
                    if (a.conj_tab) w.y = -w.y;
                    tile[e * pitch + c] = mul<T>(tile[e * pitch + c], w);
                }
            }
            __syncthreads();
        }
        if (a.inv) line_fft<T, MAXV, true, ODD>(tile, tw, a.p, pitch, 1, a.W, true, tid, nthr);

        if (a.mode == 0) {
            T* obase_ptr = a.items ? reinterpret_cast<T*>(a.items[item].out)
                                   : reinterpret_cast<T*>(a.out0) + (long long)item * a.item_stride_out;
            C<T>* out = reinterpret_cast<C<T>*>(obase_ptr + obase);
#pragma unroll 1
            for (int i0 = tid; i0 < P; i0 += STG * nthr) {
                C<T> v[STG];
#pragma unroll
                for (int k = 0; k < STG; ++k) {
                    const int i = i0 + k * nthr;
                    const int e = i / a.W;
                    if (i < P) v[k] = tile[e * pitch + (i - e * a.W)];
                }
#pragma unroll
                for (int k = 0; k < STG; ++k) {
                    const int i = i0 + k * nthr;
                    const int e = i / a.W;
                    const int c = i - e * a.W;
                    if (i < P && c0 + c < a.ncols) out[(e * astride) / 2 + c0 + c] = v[k];
                }
            }
        } else {
            T* out0 = reinterpret_cast<T*>(a.out0) + (long long)item * a.item_stride_out + obase * es;
            T* out1 = last_odd ? reinterpret_cast<T*>(a.lone_out1)
                               : (a.out1 ? reinterpret_cast<T*>(a.out1) + (long long)item * a.item_stride_out : nullptr);
            if (out1) out1 += obase * es;
#pragma unroll 1
            for (int i0 = tid; i0 < P; i0 += STG * nthr) {
                C<T> v[STG];
#pragma unroll
                for (int k = 0; k < STG; ++k) {
                    const int i = i0 + k * nthr;
                    const int e = i / a.W;
                    if (i < P) v[k] = tile[e * pitch + (i - e * a.W)];
                }
#pragma unroll
                for (int k = 0; k < STG; ++k) {
                    const int i = i0 + k * nthr;
                    const int e = i / a.W;
                    const int c = i - e * a.W;
                    if (i < P && c0 + c < a.ncols) {
                        const long long off = (e * astride + c0 + c) * es;
                        out0[off] = v[k].x;
                        if (out1) out1[off] = v[k].y;
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------ host launchers
template <typename T, int MAXV, bool ODD>
static hipError_t launch_slab_t(const SlabArgs& a, int nthr, int nblocks, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((slab_kernel<T, MAXV, ODD>), dim3(nblocks), dim3(nthr), lds, s, a);
    return hipGetLastError();
}

template <typename T, int MAXV, bool ODD, bool SHIFT = false>
static hipError_t launch_pencil_t(const PencilArgs& a, int nthr, int nblocks, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((pencil_kernel<T, MAXV, ODD, SHIFT>), dim3(nblocks), dim3(nthr), lds, s, a);
    return hipGetLastError();
}

// Lengths with a prime factor above 3 need the kernels that carry the radix-5/7
// codelets and the direct stage (kept out of the 2^a 3^b kernels, whose register
// allocation they would raise).  Those kernels take at most 512 threads.
static bool needs_odd_stages(const RadixPlan& p) {
    if (p.rader) return true;
    for (int i = 0; i < p.nst; ++i)
        if (p.r[i] != 2 && p.r[i] != 3 && p.r[i] != 4 && p.r[i] != 8 && p.r[i] != 16) return true;
    return false;
}

// Allow every pass kernel the full 160 KB of LDS (done once, outside any capture).
hipError_t prepare_generic_kernels() {
    const int lds = 160 * 1024;
    const void* fns[] = {reinterpret_cast<const void*>(slab_kernel<float, SE2C_MAXV, false>),
                         reinterpret_cast<const void*>(slab_kernel<double, SE2C_MAXV_F64, false>),
                         reinterpret_cast<const void*>(pencil_kernel<float, SE2C_MAXV, false>),
                         reinterpret_cast<const void*>(pencil_kernel<double, SE2C_MAXV_F64, false>),
                         reinterpret_cast<const void*>(slab_kernel<float, SE2C_MAXV_ODD, true>),
                         reinterpret_cast<const void*>(slab_kernel<double, SE2C_MAXV_ODD, true>),
                         reinterpret_cast<const void*>(pencil_kernel<float, SE2C_MAXV_ODD, true>),
                         reinterpret_cast<const void*>(pencil_kernel<double, SE2C_MAXV_ODD, true>),
                         reinterpret_cast<const void*>(pencil_kernel<float, SE2C_MAXV_SHIFT, false, true>),
                         reinterpret_cast<const void*>(pencil_kernel<double, SE2C_MAXV_SHIFT, false, true>),
                         reinterpret_cast<const void*>(pencil_kernel<float, SE2C_MAXV_ODD, true, true>),
                         reinterpret_cast<const void*>(pencil_kernel<double, SE2C_MAXV_ODD, true, true>)};
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t slab_lds_bytes(const SlabArgs& a, bool dbl) {
    const int cb = dbl ? 16 : 8;
    return (size_t)cb * ((size_t)a.rows_per_tile * (a.nx + a.pad) + tables_slots(a.px, cb) + tables_slots(a.pt, cb) +
                         (size_t)a.nx + (size_t)a.m);
}

size_t pencil_lds_bytes(const PencilArgs& a, bool dbl) {
    const int cb = dbl ? 16 : 8;
    return (size_t)cb * ((size_t)a.p.L * (a.W + a.pad) + tables_slots(a.p, cb) + (size_t)a.p.L);
}

hipError_t launch_slab(const SlabArgs& a, bool dbl, int nthr, int nblocks, hipStream_t s) {
    const size_t lds = slab_lds_bytes(a, dbl);
    const bool odd = needs_odd_stages(a.px) || (a.do_t && needs_odd_stages(a.pt));
    if (odd) {
        if (dbl) return launch_slab_t<double, SE2C_MAXV_ODD, true>(a, nthr, nblocks, lds, s);
        return launch_slab_t<float, SE2C_MAXV_ODD, true>(a, nthr, nblocks, lds, s);
    }
    if (dbl) return launch_slab_t<double, SE2C_MAXV_F64, false>(a, nthr, nblocks, lds, s);
    return launch_slab_t<float, SE2C_MAXV, false>(a, nthr, nblocks, lds, s);
}

hipError_t launch_pencil(const PencilArgs& a, bool dbl, int nthr, int nblocks, hipStream_t s) {
    const size_t lds = pencil_lds_bytes(a, dbl);
    if (a.mul == 3) {
        if (needs_odd_stages(a.p)) {
            if (dbl) return launch_pencil_t<double, SE2C_MAXV_ODD, true, true>(a, nthr, nblocks, lds, s);
            return launch_pencil_t<float, SE2C_MAXV_ODD, true, true>(a, nthr, nblocks, lds, s);
        }
        if (dbl) return launch_pencil_t<double, SE2C_MAXV_SHIFT, false, true>(a, nthr, nblocks, lds, s);
        return launch_pencil_t<float, SE2C_MAXV_SHIFT, false, true>(a, nthr, nblocks, lds, s);
    }
    if (needs_odd_stages(a.p)) {
        if (dbl) return launch_pencil_t<double, SE2C_MAXV_ODD, true>(a, nthr, nblocks, lds, s);
        return launch_pencil_t<float, SE2C_MAXV_ODD, true>(a, nthr, nblocks, lds, s);
    }
    if (dbl) return launch_pencil_t<double, SE2C_MAXV_F64, false>(a, nthr, nblocks, lds, s);
    return launch_pencil_t<float, SE2C_MAXV, false>(a, nthr, nblocks, lds, s);
}

}  // namespace se2c

namespace se2c {
hipError_t prepare_fast_kernels();
hipError_t prepare_fast64_kernels();
hipError_t prepare_kernels() {
    static hipError_t once = [] {
        hipError_t e = prepare_generic_kernels();
        if (e == hipSuccess) e = prepare_fast_kernels();
        if (e == hipSuccess) e = prepare_fast64_kernels();
        return e != hipSuccess ? e : prepare_full_fast_kernels();
    }();
    return once;
}
}  // namespace se2c
