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

// Multi-class launches: every shape class of a submission in one launch per pass.
#define SE2C_MULTI_THREADS 256
#define SE2C_MAX_CLASSES 16
struct MultiClass {
    int nx, ny, m;
    int nitems;          // fields of the class
    int item0;           // first of them in MultiArgs::items
    int code;            // kernel body (filled by the launcher)
    int first_block;     // first workgroup of the class (filled by the launcher)
    const float2* twx;   // FP64-generated twiddles of Nx, Ny, M (rounded)
    const float2* twy;
    const float2* twt;
    const float2* tw;    // the pass's line twiddles (filled by the launcher)
};
struct MultiArgs {
    const SepItem* items;  // device
    int conj_tab;
    int nclass;
    MultiClass c[SE2C_MAX_CLASSES];
};
bool multi_slab_supported(int nx, int m);
bool multi_pencil_supported(int nx, int ny);
hipError_t launch_slab_multi(MultiArgs m, hipStream_t s);
hipError_t launch_pencil_multi(MultiArgs m, hipStream_t s);

bool slab_fast_supported(int nx, int m);
bool pencil_fast_supported(int nx, int ny);
bool three_pass_fast_supported(int nx, int ny, int m);
hipError_t launch_slab_fast(const FastSepArgs& a, hipStream_t s);
hipError_t launch_pencil_fast(const FastSepArgs& a, hipStream_t s);
hipError_t launch_rows_fast(const FastSepArgs& a, hipStream_t s);
hipError_t prepare_fast_kernels();

}  // namespace se2c
