// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11).  Counter-based: a draw is a pure function of
// (counter, key), so any thread can produce any draw of a stream directly.
//
// Draw conventions used by the library (one block = 4 words):
//   uniform fp32 in [0,1)   (w >> 8) * 2^-24
//   uniform int in [0, N)   (w * N) >> 32
//   Bernoulli(rho)          (w >> 8) < floor(rho * 2^24)
// Counter = {word-block index, individual or slot, generation, stream tag};
// key = the 64-bit seed split into two words.
#pragma once

#include <cstdint>

namespace vrprpd {

constexpr uint32_t kTagMutant = 0x4D555441u;
constexpr uint32_t kTagParent = 0x50415245u;
constexpr uint32_t kTagCross = 0x43524F53u;
constexpr uint32_t kTagWarm = 0x5741524Du;
constexpr uint32_t kTagRandom = 0x52414E44u;

struct Philox4 {
    uint32_t x[4];
};

__host__ __device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                         uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return Philox4{{c0, c1, c2, c3}};
}

// Word (a % 4) of block {a / 4, b, c, tag} under the seed.
__host__ __device__ __forceinline__ uint32_t philox_word(uint64_t seed, uint32_t a, uint32_t b, uint32_t c,
                                                         uint32_t tag)
{
    const Philox4 r = philox4x32_10(a >> 2, b, c, tag, (uint32_t)seed, (uint32_t)(seed >> 32));
    return r.x[a & 3];
}

__host__ __device__ __forceinline__ float unit24(uint32_t w) { return (float)(w >> 8) * (1.0f / 16777216.0f); }

}  // namespace vrprpd
