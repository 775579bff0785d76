// Philox4x32-10 counter-based generator for the device, from its published
// definition (J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11): ten rounds; each round forms the
// two 64-bit products of counter words 0 and 2 with the round multipliers,
// mixes their high halves with counter words 1 and 3 and the round key, and the
// key advances by the Weyl constants between rounds.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace muca {

struct Ctr4 {
    uint32_t v[4];
};

// a ^ b ^ c in one instruction (three-input bitwise op of gfx950, truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

constexpr uint32_t kPhiloxMulA = 0xD2511F53u, kPhiloxMulB = 0xCD9E8D57u;
constexpr uint32_t kPhiloxWeylA = 0x9E3779B9u, kPhiloxWeylB = 0xBB67AE85u;

__device__ __forceinline__ Ctr4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t key0, uint32_t key1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t ka = key0 + kPhiloxWeylA * (uint32_t)round;
        const uint32_t kb = key1 + kPhiloxWeylB * (uint32_t)round;
        const uint64_t pa = (uint64_t)kPhiloxMulA * c0;
        const uint64_t pb = (uint64_t)kPhiloxMulB * c2;
        const uint32_t t0 = xor3((uint32_t)(pb >> 32), c1, ka);
        const uint32_t t2 = xor3((uint32_t)(pa >> 32), c3, kb);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = t0;
        c2 = t2;
    }
    Ctr4 r;
    r.v[0] = c0; r.v[1] = c1; r.v[2] = c2; r.v[3] = c3;
    return r;
}

// The twenty round keys (key0 + r weylA, key1 + r weylB), held in vector
// registers by a caller that runs the generator in a latency-bound loop: the
// rounds then take their keys as operands instead of rebuilding them with
// scalar adds on every call.
__device__ __forceinline__ void philox_round_keys(uint32_t key0, uint32_t key1, uint32_t (&rk)[20])
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        rk[2 * round] = key0 + kPhiloxWeylA * (uint32_t)round;
        rk[2 * round + 1] = key1 + kPhiloxWeylB * (uint32_t)round;
        asm volatile("" : "+v"(rk[2 * round]), "+v"(rk[2 * round + 1]));
    }
}

// a ^ b ^ c with all three operands in vector registers
__device__ __forceinline__ uint32_t xor3v(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// philox10 with the round keys of philox_round_keys.
__device__ __forceinline__ Ctr4 philox10_rk(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            const uint32_t (&rk)[20])
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)kPhiloxMulA * c0;
        const uint64_t pb = (uint64_t)kPhiloxMulB * c2;
        const uint32_t t0 = xor3v((uint32_t)(pb >> 32), c1, rk[2 * round]);
        const uint32_t t2 = xor3v((uint32_t)(pa >> 32), c3, rk[2 * round + 1]);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = t0;
        c2 = t2;
    }
    Ctr4 r;
    r.v[0] = c0; r.v[1] = c1; r.v[2] = c2; r.v[3] = c3;
    return r;
}

}  // namespace muca
