// phase.hpp -- device representation of oscillator phases.
//
// A phase is held as a 32-bit fixed-point fraction of a turn,
// u = theta / 2pi * 2^32 (mod 2^32), like the phase accumulator of a
// numerically controlled oscillator.  The wrap of Algorithm 1 (the phase
// normalised to one turn) is then exact integer overflow, and the state resolution is
// 2^-32 turn (1.5e-9 rad) instead of FP32's 4.8e-7 rad near 2pi, so rounding
// of the state no longer accumulates over the steps.  All dynamics arithmetic
// stays FP32: increments are computed in FP32 in units of 2^-32 turn and
// rounded to the nearest integer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oim {

constexpr double kTwoPiD = 6.283185307179586476925286766559;
constexpr float kTurnScale = 683565275.57643158978045f;  // 2^32 / 2pi

// Signed turn fraction in [-1/2, 1/2) as FP32 (best argument for v_sin/v_cos,
// which take revolutions).
__device__ __forceinline__ float turns(uint32_t u) {
    return (float)(int32_t)u * 0x1.0p-32f;
}

__device__ __forceinline__ float sin_turn(uint32_t u) { return __builtin_amdgcn_sinf(turns(u)); }
__device__ __forceinline__ float cos_turn(uint32_t u) { return __builtin_amdgcn_cosf(turns(u)); }

// Advance by an FP32 increment expressed in 2^-32 turn units.
__device__ __forceinline__ uint32_t advance(uint32_t u, float du) {
    return u + (uint32_t)(int32_t)__builtin_rintf(du);
}

// Radians -> phase word, FP64 conversion; a non-finite phase (NaN, +-Inf)
// is taken as 0.
__device__ __forceinline__ uint32_t phase_from_theta(float th) {
    if (!__builtin_isfinite(th)) return 0u;
    const double x = (double)th / kTwoPiD;
    const double f = x - __builtin_floor(x);                      // [0, 1]
    const double w = __builtin_rint(f * 4294967296.0);             // [0, 2^32]
    return (uint32_t)(uint64_t)w;                                  // 2^32 wraps to 0
}

// Phase word -> radians in [0, 2pi) as FP32 (correctly rounded, clamped below 2pi).
__device__ __forceinline__ float theta_from_phase(uint32_t u) {
    float t = (float)((double)u * (kTwoPiD / 4294967296.0));
    return t < 6.2831854820251465f ? t : 6.2831850051879883f;   // (float)2pi -> next below
}

// Nearest stable phase index floor(q u / 2^32 + 1/2) mod q, exact.
__device__ __forceinline__ int nearest_state(uint32_t u, int q) {
    const uint32_t k = (uint32_t)(((uint64_t)q * u + 0x80000000ull) >> 32);
    return k >= (uint32_t)q ? 0 : (int)k;
}

// sin(q theta) from the phase word (generic q) or from (sin, cos) for q = 2, 3.
template <int QM>
__device__ __forceinline__ float sin_q(float s, float c, uint32_t u, int q) {
    if constexpr (QM == 2) {
        return 2.0f * s * c;
    } else if constexpr (QM == 3) {
        return s * (3.0f - 4.0f * s * s);
    } else {
        return sin_turn((uint32_t)q * u);
    }
}

}  // namespace oim
