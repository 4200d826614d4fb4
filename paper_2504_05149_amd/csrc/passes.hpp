// Host-visible argument blocks and launchers of the pass kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "fft_device.hpp"
#include "shift.hpp"

#define SE2C_MAXV 16          // complex values held per thread during a stage
// The same for the kernels with radix-5/7, direct and Rader stages: a smaller budget
// keeps their register allocation low enough for several workgroups per CU.
#ifndef SE2C_MAXV_ODD
#define SE2C_MAXV_ODD 8
#endif
// The same for the FP64 kernels without odd stages (8 measured faster than 16 and 4
// at 512x512x128).
#ifndef SE2C_MAXV_F64
#define SE2C_MAXV_F64 8
#endif
// The same for the pencils that carry the shift mix (they hold a second copy of their
// values while the mix reads rolled neighbours).
#ifndef SE2C_MAXV_SHIFT
#define SE2C_MAXV_SHIFT 8
#endif
// Tile elements per thread whose HBM reads are in flight together when a tile is
// loaded or stored.
#ifndef SE2C_STAGE
#define SE2C_STAGE 4
#endif
#define SE2C_MAX_TABLES 8     // kernels multiplied at run time in one pass
// Threads per workgroup: FP32 tiles use up to 1024 (128 VGPRs each), FP64 tiles
// up to 512 so that the doubled register footprint does not spill.
#define SE2C_MAX_THREADS(T) (sizeof(T) == 8 ? 512 : 1024)

namespace se2c {

// One field of a heterogeneous launch (separable tables only): its input, output
// and the SEPARABLE tables of its chain (Tx at 0, Ty at Nx, Tt at Nx + Ny complex).
// Slab passes read `in` and write `out`; pencil passes run in place on `out`.
struct SepItem {
    const void* in;
    void* out;
    const void* tab[SE2C_MAX_TABLES];
    int ntab;
};

// Tile = rows_per_tile theta-rows x nx of one y-slab.  in_mode/out_mode:
// 0 = y-pair of one real field (rows 2s, 2s+1), 1 = two real planes (in0, in1).
struct SlabArgs {
    const void* in0;
    const void* in1;
    void* out0;
    void* out1;
    const void* lone_in1;   // plane mode: imaginary input of the last item when the count is odd
    void* lone_out1;        // plane mode: imaginary output of the last item (nullptr = drop)
    long long item_stride_in;
    long long item_stride_out;
    int nitems;
    int in_mode, out_mode;
    int nx, ny, m;
    int rows_per_tile;
    int ntile_t;            // theta chunks per slab
    int nslab;              // slabs per item
    int pad;                // LDS row padding (complex)
    int do_t;               // also transform along theta (requires rows_per_tile == m)
    int fwd, inv;
    int mul;                // 1: separable product with ntab tables (factors x [and theta])
    int ntab;
    const void* tx[SE2C_MAX_TABLES];
    const void* tt[SE2C_MAX_TABLES];
    int conj_tab;
    double scale;
    RadixPlan px, pt;
    const void* twx;
    const void* twt;
    const SepItem* items;   // device; non-null: item i reads items[i] (y-pair modes, separable product)
    int cplx;               // plane mode: planes are interleaved (complex fields; in1 = in0 + 1, element stride 2)
};

// Tile = W adjacent columns x L points along axis (1 = y, 2 = theta) at a fixed
// other coordinate.  mode 0 = x-pair view of one real field, 1 = two real planes.
struct PencilArgs {
    const void* in0;
    const void* in1;
    void* out0;
    void* out1;
    const void* lone_in1;
    void* lone_out1;
    long long item_stride_in;
    long long item_stride_out;
    int nitems;
    int mode;
    int axis;
    int nx, ny, m;
    int ncols;
    int W;
    int pad;
    int fwd, inv;
    int mul;                // 1: 1-D factors (sep tables), 2: full tables / mixed, 3: as 2 along theta,
                            // after the shift mix before the forward transform (qtab, rolls)
    int ntab;
    const void* tab1[SE2C_MAX_TABLES];    // 1-D factor along this axis (mul == 1)
    const void* tab3[SE2C_MAX_TABLES];    // full [m][ny][nx] table, or nullptr if separable
    unsigned tab3_quarter;                // bit j: tab3[j] is a quarter table [m][ny/2+1][nx/2+1]
    const void* sepx[SE2C_MAX_TABLES];    // separable factors for mul == 2 with sep tables
    const void* sepy[SE2C_MAX_TABLES];
    const void* sept[SE2C_MAX_TABLES];
    int conj_tab;
    double scale;
    RadixPlan p;
    const void* tw;
    const SepItem* items;   // device; non-null: item i reads items[i] (x-pair mode, 1-D factor product)
    int cplx;               // plane mode: planes are interleaved (complex fields; in1 = in0 + 1, element stride 2)
    // mul == 3 (theta lines of spatial spectra): before the forward transform every point
    // alpha becomes sum_j z[alpha - rolls[j]] Q_j[alpha - rolls[j]][k2][k1] (indices mod M),
    // Q_j the j-th [M][Ny][Nx] complex plane set of qtab
    const void* qtab;
    int nshift;
    int rolls[SE2C_MAX_SHIFT_CLASSES];
};

size_t slab_lds_bytes(const SlabArgs& a, bool dbl);
size_t pencil_lds_bytes(const PencilArgs& a, bool dbl);
hipError_t launch_slab(const SlabArgs& a, bool dbl, int nthr, int nblocks, hipStream_t s);
hipError_t launch_pencil(const PencilArgs& a, bool dbl, int nthr, int nblocks, hipStream_t s);
// Register pencils (FP32 / FP64) for the prime lengths rader_fast_supported lists
// (rader_fast.hip): planes of field pairs (mode 1, no per-item tables); forward + product
// (mul 2) + inverse along y or theta, or one direction alone (mul 0, also x rows: axis 0).
// hipErrorInvalidValue for anything else.
bool rader_fast_supported(int L, bool dbl);
hipError_t launch_rader_pencil(const PencilArgs& a, bool dbl, hipStream_t s);

// Raise the dynamic-LDS limit of the pass kernels (call once before any capture).
hipError_t prepare_generic_kernels();
hipError_t prepare_kernels();

// Zero-padded spectra of nitems field pairs: L-grid planes -> G-grid planes, G >= L per
// axis (pad.hip).
hipError_t launch_pad_spectrum(const void* src, void* dst, void* lone, int nitems, long long src_stride,
                               long long dst_stride, int lx, int ly, int lm, int gx, int gy, int gm, bool dbl,
                               hipStream_t s);

// FP64 twiddles w_L^j = exp(-2 pi i j / L), j in [0, L), written as double2 and float2.
hipError_t launch_twiddles(double2* out64, float2* out32, int L, hipStream_t s);

}  // namespace se2c
