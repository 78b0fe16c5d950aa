// noise.hpp -- device-side Gaussian noise for the Euler-Maruyama step
// (Sec. II-E Eq. 5 eta_i(t); Algorithm 1 "noise" line).
//
// The paper draws from per-thread cuRAND states.  Here the stream is
// stateless and counter-based so any (replica, oscillator, step) can be
// regenerated without stored generator state:
//   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): two 32x32->64 products
//   per round, multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key increments
//   0x9E3779B9 / 0xBB67AE85, ten rounds.
//   key     = (seed & 0xffffffff, seed >> 32)
//   counter = (i >> 2, t, b, 0)      t = global step index, i the oscillator's
//                                    index within its instance, b the instance
//                                    of a block-diagonal batch (0 otherwise)
//   one call gives the normals of oscillators 4m..4m+3 via Box-Muller
//   (Box & Muller 1958) on the word pairs (x0,x1) and (x2,x3):
//   u1 = ((xa >> 8) + 1) * 2^-24 in (0,1], u2 = (xb >> 8) * 2^-24 in [0,1),
//   rho = sqrt(-2 ln u1), z_even = rho cos(2 pi u2), z_odd = rho sin(2 pi u2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oim {

struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ void philox_mulhilo(uint32_t m, uint32_t a, uint32_t& hi, uint32_t& lo) {
    const uint64_t p = (uint64_t)m * (uint64_t)a;
    hi = (uint32_t)(p >> 32);
    lo = (uint32_t)p;
}

// Ten Philox rounds on counter c with key (k0, k1).
__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0, lo0, hi1, lo1;
        philox_mulhilo(0xD2511F53u, c.x, hi0, lo0);
        philox_mulhilo(0xCD9E8D57u, c.z, hi1, lo1);
        c = u32x4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Box-Muller on one word pair, FP32, with the hardware transcendentals:
// v_log_f32 is log2, v_sin/v_cos take revolutions (so 2 pi u2 needs no
// multiply).  Writes the even (cos) and odd (sin) member of the pair.
__device__ __forceinline__ void box_muller(uint32_t xa, uint32_t xb, float& z_even, float& z_odd) {
    const float u1 = __builtin_fmaf((float)(xa >> 8), 0x1.0p-24f, 0x1.0p-24f);
    const float u2 = (float)(xb >> 8) * 0x1.0p-24f;
    // -2 ln u1 = -2 ln(2) log2(u1)
    const float rho = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u1));
    z_even = rho * __builtin_amdgcn_cosf(u2);
    z_odd = rho * __builtin_amdgcn_sinf(u2);
}

// The four normals of oscillators 4m..4m+3 of instance b at step t for a
// replica key.
__device__ __forceinline__ void normals4(uint32_t m, uint32_t t, uint32_t b, uint32_t k0,
                                         uint32_t k1, float z[4]) {
    const u32x4 x = philox4x32_10(u32x4{m, t, b, 0u}, k0, k1);
    box_muller(x.x, x.y, z[0], z[1]);
    box_muller(x.z, x.w, z[2], z[3]);
}

// The two normals of one word pair (pair 0: oscillators 4m, 4m+1; pair 1:
// 4m+2, 4m+3) of the same Philox call, bit-identical to those normals4
// returns for them.
__device__ __forceinline__ void normals2(uint32_t m, uint32_t t, uint32_t b, uint32_t k0,
                                         uint32_t k1, int pair, float z[2]) {
    const u32x4 x = philox4x32_10(u32x4{m, t, b, 0u}, k0, k1);
    box_muller(pair ? x.z : x.x, pair ? x.w : x.y, z[0], z[1]);
}

}  // namespace oim
