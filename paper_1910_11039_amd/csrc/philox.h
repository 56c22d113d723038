// Philox4x64-10 counter-based generator on the device, from its published
// definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11): ten rounds of two 64x64->128 multiplications with the
// Philox multipliers, Weyl key schedule in between.
//
// Stream layout used by the sampler: key = (seed, stream), counter =
// (block, sample index, 0, 0); draw j of a sample is word j mod 4 of
// block floor(j / 4).  Draw 0 and 1 pick the pair, draw 2 the meet vertex,
// draws 3, 4, ... the predecessors while walking back.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kad {

__device__ __forceinline__ void philox4x64_10(uint64_t k0, uint64_t k1, uint64_t c[4])
{
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0;
        const uint64_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

// Draws of one sample; caches the last block (wave-uniform use).
struct SampleDraws {
    uint64_t seed, stream, sample;
    uint64_t blk;
    uint64_t w[4];

    __device__ void init(uint64_t sd, uint64_t sm, uint64_t idx)
    {
        seed = sd;
        stream = sm;
        sample = idx;
        blk = ~0ull;
    }

    __device__ uint64_t get(uint64_t j)
    {
        const uint64_t b = j >> 2;
        if (b != blk) {
            w[0] = b;
            w[1] = sample;
            w[2] = 0;
            w[3] = 0;
            philox4x64_10(seed, stream, w);
            blk = b;
        }
        switch (j & 3) {
        case 0: return w[0];
        case 1: return w[1];
        case 2: return w[2];
        default: return w[3];
        }
    }
};

}  // namespace kad
