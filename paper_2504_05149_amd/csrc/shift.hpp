// Translation-phase tables of kernels that are sums of SE(2)-shifts of one kernel
// radial in translations (see shift.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace se2c {

#define SE2C_MAX_SHIFT_TERMS 64   // shifts per table
#define SE2C_MAX_SHIFT_CLASSES 8  // distinct theta rolls per table

struct ShiftTerm {
    double tx, ty;  // translation t of the shift
    double w;       // weight a_k
};

// Terms of one roll class: their translation phases are summed into one plane set.
struct ShiftClassArgs {
    int nx, ny, m;
    int nterm;
    ShiftTerm t[SE2C_MAX_SHIFT_TERMS];
};

// Q[alpha][t2][t1] = sum_terms w E_x(t1; (R_alpha t)_x) E_y(t2; (R_alpha t)_y) of one class,
// evaluated in FP64 and stored rounded once (FP32 complex when dbl == 0, else FP64).
hipError_t launch_shift_table(const ShiftClassArgs& a, void* out, bool dbl, hipStream_t s);

}  // namespace se2c
