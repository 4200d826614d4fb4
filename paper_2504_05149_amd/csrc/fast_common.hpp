// Device helpers shared by the register-resident FP32 pass kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "fft_device.hpp"

namespace se2c {

// Position of element (k1, t) of one R1 x R2 exchange line (R1 = 16 or 32 values per
// thread, R2 threads per line, CC = R1 / R2 first-stage frequencies per thread after
// the exchange): the XOR swizzle makes both the write (fixed k1, lanes over t) and
// the read (fixed t, lanes over the k1 groups) hit distinct 8-byte bank slots.
template <int R1, int R2>
__device__ __forceinline__ int xpos_line(int k1, int t) {
    constexpr int CC = R1 / R2;
    return k1 * R2 + (t ^ (k1 / CC));
}
template <int R2>
__device__ __forceinline__ int xpos(int k1, int t) {
    return xpos_line<16, R2>(k1, t);
}

// Synchronisation of the lanes of one wavefront around an LDS exchange among them:
// release / acquire fences at wavefront scope and a wave barrier, so neither the
// compiler nor the hardware moves this wave's LDS reads ahead of its earlier writes.
// Used where every line of an exchange lives in one wavefront (R2 <= 16 consecutive
// lanes), instead of a workgroup barrier.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// scale * prod_j tabs[j][i] (conjugated for the adjoint)
__device__ __forceinline__ float2 chain_factor(const void* const* tabs, int ntab, int i, float scale, int conj) {
    float2 v = make_float2(scale, 0.f);
    for (int j = 0; j < ntab; ++j) v = mul<float>(v, reinterpret_cast<const float2*>(tabs[j])[i]);
    if (conj) v.y = -v.y;
    return v;
}

// The same, with the tables given by an accessor tab(j) -> const float2* (no local array
// of table pointers, which a dynamic index would place in scratch memory).
template <typename F>
__device__ __forceinline__ float2 chain_factor_of(F tab, int ntab, int i, float scale, int conj) {
    float2 v = make_float2(scale, 0.f);
    for (int j = 0; j < ntab; ++j) v = mul<float>(v, tab(j)[i]);
    if (conj) v.y = -v.y;
    return v;
}

// Swap a value with the neighbouring lane (lane ^ 1) through DPP quad_perm [1,0,3,2].
__device__ __forceinline__ float swap_lane1(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ float2 swap_lane1(float2 v) { return make_float2(swap_lane1(v.x), swap_lane1(v.y)); }

}  // namespace se2c
