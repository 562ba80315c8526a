// gm_philox.h -- Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11) for the
// device code of the library: ten rounds of two 32x32 -> 64-bit products whose
// high halves are mixed with the odd counter words and the round key, the key
// advancing by two Weyl increments between rounds.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gm {

__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                              uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t hi_a = __umulhi(0xD2511F53u, c0), lo_a = 0xD2511F53u * c0;
        const uint32_t hi_b = __umulhi(0xCD9E8D57u, c2), lo_b = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi_b ^ c1 ^ k0;
        const uint32_t n2 = hi_a ^ c3 ^ k1;
        c0 = n0; c1 = lo_b; c2 = n2; c3 = lo_a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

}  // namespace gm
