// Philox-4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11),
// usable on host and device.  Float mapping convention of this library:
//   u = (w >> 8) * 2^-24 + 2^-25 in (0, 1);
//   normal pair by Box-Muller: sqrt(-2 ln u0) * (cos 2 pi u1, sin 2 pi u1).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace helm {

struct u32x4 {
    uint32_t v[4];
};

__host__ __device__ inline u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
    const uint64_t M0 = 0xD2511F53ull, M1 = 0xCD9E8D57ull;
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = M0 * (uint64_t)c.v[0];
        uint64_t p1 = M1 * (uint64_t)c.v[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        u32x4 n;
        n.v[0] = hi1 ^ c.v[1] ^ k0;
        n.v[1] = lo1;
        n.v[2] = hi0 ^ c.v[3] ^ k1;
        n.v[3] = lo0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__host__ __device__ inline double philox_u01(uint32_t w) {
    return (double)(w >> 8) * (1.0 / 16777216.0) + (1.0 / 33554432.0);
}

// Entry i of stream s, key (k0,k1): words of counter (i, s, 0, 0).
__host__ __device__ inline u32x4 philox_at(uint64_t i, uint32_t s, uint32_t k0, uint32_t k1) {
    u32x4 c;
    c.v[0] = (uint32_t)i;
    c.v[1] = s;
    c.v[2] = 0;
    c.v[3] = 0;
    return philox4x32_10(c, k0, k1);
}

}  // namespace helm
