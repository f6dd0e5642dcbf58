// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11) and the stream
// layout of this library: domain in bits 24..31 of the third counter word.
// Usable from host and device code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sg {

enum : uint32_t { kDomSweepHi = 0, kDomSweepLo = 1, kDomInit = 2, kDomGraph = 3, kDomCoupling = 4 };

struct U4 {
    uint32_t x, y, z, w;
};

__host__ __device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t b = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
#if defined(__HIP_DEVICE_COMPILE__)
        // three-input XOR in one gfx950 VALU instruction (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(b >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), c3, k1, 0x96);
#else
        const uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
#endif
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

__host__ __device__ __forceinline__ U4 philox_stream(uint64_t seed, uint32_t c0, uint32_t c1,
                                                     uint32_t dom, uint32_t sub, uint32_t c3)
{
    return philox10(c0, c1, (dom << 24) | sub, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// Half-word h (0..7) of a block.
__host__ __device__ __forceinline__ uint32_t half_word(const U4& w, uint32_t h)
{
    const uint32_t q = h >> 1;
    const uint32_t word = q == 0 ? w.x : q == 1 ? w.y : q == 2 ? w.z : w.w;
    return (word >> (16u * (h & 1u))) & 0xffffu;
}

__host__ __device__ __forceinline__ uint32_t word_of(const U4& w, uint32_t q)
{
    return q == 0 ? w.x : q == 1 ? w.y : q == 2 ? w.z : w.w;
}

}  // namespace sg
