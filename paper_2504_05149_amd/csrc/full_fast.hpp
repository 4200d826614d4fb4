// Register-resident FP32 kernels of the full-table (non-separable) path (see full_fast.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "passes.hpp"

namespace se2c {

// Fields are processed in pairs packed as re/im: pair p is fields 2p (re) and 2p + 1
// (im).  Its x-theta spectrum occupies the two field slots as real planes (re plane
// in slot 2p, im plane in slot 2p + 1); with an odd batch the last pair's im plane
// lives in `lone` (one plane of workspace).
struct FullFastArgs {
    const float* in;
    float* out;
    float* lone;            // im plane of the last pair when the batch is odd (else unused)
    long long n;            // points per field
    int batch;              // fields
    int nx, ny, m;
    const float2* twx;      // w_nx^j
    const float2* twy;      // w_ny^j
    const float2* twt;      // w_m^j
    // y pass: product with scale * prod_j T_j (FULL: [m][ny][nx]; SEPARABLE: Tx Ty Tt)
    int ntab;
    const void* tab[SE2C_MAX_TABLES];
    int tab_full[SE2C_MAX_TABLES];  // 1 FULL [m][ny][nx], 2 quarter [m][ny/2+1][nx/2+1], 0 SEPARABLE
    float scale;
    int conj_tab;
    float* save;            // y pass: if non-null, the spectrum before the product goes to
                            // save (slots 2p, 2p + 1 per pair, planes as above)
    float* save_lone;       // if non-null, slot 2p + 1 of a lone last field goes here instead
                            // (save == out in place: the lone field's im plane, as lone)
    // backward y pass
    const float* zf;        // field spectra (slots 2p, 2p + 1 per pair)
    float* acc;             // two planes: W A / n^2 after the inverse DFT along y
    float acc_scale;        // 1 / n^2
    // powers y pass: q output slots of batch fields each, `slot` reals apart, starting at out
    int q;
    long long slot;
    // evaluation on a finer grid: the y spectra on the sampling grid (lx, ly, lm; nl points
    // per plane, two planes per pair) that the y pass of the evaluation grid pads and inverts;
    // the tables belong to the sampling grid
    const float* zsrc;
    int lx, ly, lm;
    long long nl;
    // shift-mix theta pass: alpha becomes sum_j z[alpha - rolls[j]] Q_j[alpha - rolls[j]][ky][kx]
    // (indices mod m), Q_j the j-th [m][ny][nx] complex plane set of qtab
    const float2* qtab;
    int nshift;
    int rolls[SE2C_MAX_SHIFT_CLASSES];
};

bool full_fast_supported(int nx, int ny, int m);
// x-theta forward DFT of field pairs (in: fields, out: spectrum planes; may alias)
hipError_t launch_xt_full_fwd(const FullFastArgs& a, hipStream_t s);
// x-theta inverse DFT (in: spectrum planes, out: fields; may alias), no scaling
hipError_t launch_xt_full_inv(const FullFastArgs& a, hipStream_t s);
// forward DFT along x only (in: fields, out: re/im planes of each pair, theta in space)
hipError_t launch_x_full_fwd(const FullFastArgs& a, hipStream_t s);
// y pass in place on the spectrum planes of every pair: forward DFT, [save], product, inverse
hipError_t launch_y_full(const FullFastArgs& a, hipStream_t s);
// y pass: forward DFT only, written to save
hipError_t launch_y_full_spectra(const FullFastArgs& a, hipStream_t s);
// y pass: inverse DFT along y only, in place on the planes (the inverse of the spectra pass
// with save = out)
hipError_t launch_y_full_inverse(const FullFastArgs& a, hipStream_t s);
// theta pass of a shifted-kernel sum on the x-y spectrum planes (theta in space), in place:
// shift mix, forward DFT along theta, product with the chain; false when this (m, nshift) is
// not supported (the caller takes the generic pencils)
bool t_shift_supported(int nx, int m, int nshift);
hipError_t launch_t_shift(const FullFastArgs& a, hipStream_t s);
// y pass of the backward: adjoint product in place, kernel-sample gradient accumulated to acc
hipError_t launch_y_full_backward(const FullFastArgs& a, hipStream_t s);
// y pass of all powers (Alg. 7): forward DFT of the spectrum planes in the last slot, then
// for p = 1..q the running product with the table and its inverse, into slot p - 1
// (even batch)
hipError_t launch_y_full_powers(const FullFastArgs& a, hipStream_t s);
// y pass on the evaluation grid of a padded evaluation: product of the sampling-grid spectra
// (zsrc) with the table, zero padding to this grid and inverse DFT along y (even batch)
hipError_t launch_y_full_pad_inv(const FullFastArgs& a, hipStream_t s);
hipError_t prepare_full_fast_kernels();

}  // namespace se2c
