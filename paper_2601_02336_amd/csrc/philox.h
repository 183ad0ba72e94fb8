// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two
// 32x32->64 multiplies with the published multipliers and Weyl key schedule.
// Streams: key = run seed, counter = (index, particle, iteration, purpose).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smcgw {

enum { RNG_MOMENTUM = 1, RNG_DOUBLING = 2, RNG_LEAF = 3, RNG_RESAMPLE = 4, RNG_RECYCLE = 5 };

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Two doubles in [0, 1) with 53 random bits each from one Philox block.
__device__ __forceinline__ void rng_uniform2(uint64_t seed, uint32_t index, uint32_t particle, uint64_t iteration,
                                             uint32_t purpose, double& u0, double& u1) {
    uint32_t o[4];
    philox4x32_10(index, particle, (uint32_t)iteration, purpose, (uint32_t)seed, (uint32_t)(seed >> 32), o);
    const double s = 1.1102230246251565404e-16;  // 2^-53
    u0 = ((double)(o[0] >> 5) * 67108864.0 + (double)(o[1] >> 6)) * s;
    u1 = ((double)(o[2] >> 5) * 67108864.0 + (double)(o[3] >> 6)) * s;
}

}  // namespace smcgw
