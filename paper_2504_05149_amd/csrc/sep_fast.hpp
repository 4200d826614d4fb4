// Register-resident FP32 kernels for separable tables (see sep_fast.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "passes.hpp"

namespace se2c {

struct FastSepArgs {
    const float* in;
    float* out;
    long long n;      // real elements per field
    int nitems;       // fields
    int nx, ny, m;
    int ntab;
    const void* tx[SE2C_MAX_TABLES];
    const void* ty[SE2C_MAX_TABLES];
    const void* tt[SE2C_MAX_TABLES];
    int conj_tab;
    const float2* tw;  // FP64-generated twiddles w_L^j of the transform length (rounded)
    const float2* twt; // FP64-generated twiddles w_M^j (theta), used by the split-column slab
    int grid_blocks;   // persistent-grid size for the pencil kernel
    int cus;           // compute units of the device
    int axis;          // pencil kernel: 1 = lines along y, 2 = lines along theta
    const SepItem* items;  // device; non-null: field i is items[i] (own input, output and tables)
};

bool slab_fast_supported(int nx, int m);
bool pencil_fast_supported(int nx, int ny);
bool three_pass_fast_supported(int nx, int ny, int m);
hipError_t launch_slab_fast(const FastSepArgs& a, hipStream_t s);
hipError_t launch_pencil_fast(const FastSepArgs& a, hipStream_t s);
hipError_t launch_rows_fast(const FastSepArgs& a, hipStream_t s);
hipError_t prepare_fast_kernels();

}  // namespace se2c
