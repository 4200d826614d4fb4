// Register-resident FP64 kernels for separable tables (see sep_fast64.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "passes.hpp"

namespace se2c {

struct Fast64Args {
    const double* in;
    double* out;
    long long n;        // real elements per field
    int nitems;         // fields
    int nx, ny, m;
    int axis;           // pencils: 1 = lines along y, 2 = lines along theta
    int ntab;
    const void* tab[SE2C_MAX_TABLES];  // this pass' 1-D factors (complex double), one per table
    int conj_tab;
    const double2* tw;  // FP64 twiddles w_L^j of the pass' line length
};

bool fast64_supported(int nx, int ny, int m);
hipError_t launch_rows_f64(const Fast64Args& a, hipStream_t s);
hipError_t launch_pencil_f64(const Fast64Args& a, hipStream_t s);
hipError_t prepare_fast64_kernels();

}  // namespace se2c
