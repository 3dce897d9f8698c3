// philox.hpp -- Philox4x32-10 counter-based generator for device code.
//
// Definition: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11. Ten rounds of
//   (x0, x1, x2, x3) <- (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1, lo(M0 x0))
// with the key advanced by the Weyl constants between rounds.
//
// Streams of the optimiser: counter word 3 = (instance << 8) | tag.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qpm {

enum : uint32_t { kTagInit = 1, kTagDeIdx = 2, kTagDeCr = 3, kTagGwo = 4, kTagDgwo = 5 };

struct U4 {
    uint32_t x, y, z, w;
};

// three-input exclusive or in one VALU instruction (truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// One round is two 32 x 32 -> 64-bit multiplies (v_mad_u64_u32) and two
// three-input xors; the round keys are wave-uniform (scalar registers).
__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                       uint32_t k1)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = static_cast<uint64_t>(kMulA) * c0;
        const uint64_t pb = static_cast<uint64_t>(kMulB) * c2;
        const uint32_t n0 = xor3(static_cast<uint32_t>(pb >> 32), c1, k0);
        const uint32_t n2 = xor3(static_cast<uint32_t>(pa >> 32), c3, k1);
        c1 = static_cast<uint32_t>(pb);
        c3 = static_cast<uint32_t>(pa);
        c0 = n0;
        c2 = n2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return U4{c0, c1, c2, c3};
}

// floor(u * m / 2^32): an index in [0, m)
__host__ __device__ __forceinline__ uint32_t bounded(uint32_t u, uint32_t m)
{
    return static_cast<uint32_t>((static_cast<uint64_t>(u) * m) >> 32);
}

// (u >> 8) 2^-24 in [0, 1), exact in binary32
__device__ __forceinline__ float unit24(uint32_t u) { return static_cast<float>(u >> 8) * 0x1p-24f; }

// (u >> 8) 2^-23 - 1 in [-1, 1), exact in binary32
__device__ __forceinline__ float sym24(uint32_t u) { return static_cast<float>(u >> 8) * 0x1p-23f - 1.0f; }

}  // namespace qpm
