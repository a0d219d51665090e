// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter-based random words,
// shared by the x samplers, the learned-proposal sampler and the preconditioning
// circuit generator.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pw {

__host__ __device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = (uint32_t)p1;
        c[2] = n2;
        c[3] = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Two 64-bit words of the block with counter (g_lo, g_hi, a, stream) and key seed.
__host__ __device__ inline void philox_words(uint64_t seed, uint64_t g, uint32_t a, uint32_t stream, uint64_t& W0,
                                             uint64_t& W1) {
    uint32_t c[4] = {(uint32_t)g, (uint32_t)(g >> 32), a, stream};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    W0 = ((uint64_t)c[1] << 32) | c[0];
    W1 = ((uint64_t)c[3] << 32) | c[2];
}

constexpr uint32_t STREAM_UNIFORM = 0x554E4946u;   // "UNIF"
constexpr uint32_t STREAM_MARGINAL = 0x4D415247u;  // "MARG"
constexpr uint32_t STREAM_MADE = 0x4D414445u;      // "MADE"
constexpr uint32_t STREAM_MIX = 0x4D495843u;       // "MIXC"
constexpr uint32_t STREAM_CLIF = 0x434C4946u;      // "CLIF"

}  // namespace pw
