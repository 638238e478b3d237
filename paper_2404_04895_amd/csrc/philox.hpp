// Device-side counter-based generator for the AdaIR deviates (Sec. 2.4).
//
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  In the construct loop
// the key and three of the four counter words -- step, ant, iteration -- are
// the same for the whole wavefront, and only the city-block word varies by
// lane, so the compiler keeps the key schedule and the uniform half of the
// first round in scalar registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aco {

struct PhiloxOut {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ PhiloxOut philox10(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                             uint32_t k0, uint32_t k1) {
    constexpr uint32_t kMulA = 0xD2511F53u;  // round multiplier for word 0
    constexpr uint32_t kMulB = 0xCD9E8D57u;  // round multiplier for word 2
    constexpr uint32_t kBumpA = 0x9E3779B9u; // key schedule increments
    constexpr uint32_t kBumpB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = static_cast<uint64_t>(x0) * kMulA;
        const uint64_t pb = static_cast<uint64_t>(x2) * kMulB;
        const uint32_t rk0 = k0 + static_cast<uint32_t>(r) * kBumpA;
        const uint32_t rk1 = k1 + static_cast<uint32_t>(r) * kBumpB;
        x0 = static_cast<uint32_t>(pb >> 32) ^ x1 ^ rk0;
        x1 = static_cast<uint32_t>(pb);
        x2 = static_cast<uint32_t>(pa >> 32) ^ x3 ^ rk1;
        x3 = static_cast<uint32_t>(pa);
    }
    return PhiloxOut{x0, x1, x2, x3};
}

// Three-input XOR in one gfx950 VALU instruction (v_bitop3_b32 with truth
// table 0x96 = a ^ b ^ c, which is symmetric in its operands).  c is the
// wave-uniform round key and is read from a scalar register.
__device__ __forceinline__ uint32_t xor3_vvs(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

// Philox4x32-10 for the counter (block, step, ant, iter) of the construct
// loop, where only `block` differs between lanes.  Rounds 1 and 2 are left to
// the compiler, which evaluates their wave-uniform halves on the scalar unit;
// from round 3 on all four words differ by lane and each new word 0 / word 2
// is one 32x32->64 multiply plus one three-input XOR.
__device__ __forceinline__ PhiloxOut philox10_block(uint32_t block, uint32_t step, uint32_t ant,
                                                   uint32_t iter, uint32_t k0, uint32_t k1) {
    constexpr uint32_t kMulA = 0xD2511F53u;
    constexpr uint32_t kMulB = 0xCD9E8D57u;
    constexpr uint32_t kBumpA = 0x9E3779B9u;
    constexpr uint32_t kBumpB = 0xBB67AE85u;
    uint32_t x0 = block, x1 = step, x2 = ant, x3 = iter;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const uint64_t pa = static_cast<uint64_t>(x0) * kMulA;
        const uint64_t pb = static_cast<uint64_t>(x2) * kMulB;
        const uint32_t rk0 = k0 + static_cast<uint32_t>(r) * kBumpA;
        const uint32_t rk1 = k1 + static_cast<uint32_t>(r) * kBumpB;
        x0 = static_cast<uint32_t>(pb >> 32) ^ (x1 ^ rk0);
        x1 = static_cast<uint32_t>(pb);
        x2 = static_cast<uint32_t>(pa >> 32) ^ (x3 ^ rk1);
        x3 = static_cast<uint32_t>(pa);
    }
    // after round 2, word 3 (low half of word 0 times kMulA, word 0 being
    // uniform after round 1) is still uniform: fold it into the key first.
    {
        const uint64_t pa = static_cast<uint64_t>(x0) * kMulA;
        const uint64_t pb = static_cast<uint64_t>(x2) * kMulB;
        const uint32_t n0 = xor3_vvs(static_cast<uint32_t>(pb >> 32), x1, k0 + 2u * kBumpA);
        const uint32_t n2 = static_cast<uint32_t>(pa >> 32) ^ (x3 ^ (k1 + 2u * kBumpB));
        x0 = n0;
        x1 = static_cast<uint32_t>(pb);
        x2 = n2;
        x3 = static_cast<uint32_t>(pa);
    }
#pragma unroll
    for (int r = 3; r < 10; ++r) {
        const uint64_t pa = static_cast<uint64_t>(x0) * kMulA;
        const uint64_t pb = static_cast<uint64_t>(x2) * kMulB;
        const uint32_t n0 = xor3_vvs(static_cast<uint32_t>(pb >> 32), x1,
                                     k0 + static_cast<uint32_t>(r) * kBumpA);
        const uint32_t n2 = xor3_vvs(static_cast<uint32_t>(pa >> 32), x3,
                                     k1 + static_cast<uint32_t>(r) * kBumpB);
        x0 = n0;
        x1 = static_cast<uint32_t>(pb);
        x2 = n2;
        x3 = static_cast<uint32_t>(pa);
    }
    return PhiloxOut{x0, x1, x2, x3};
}

// Philox4x32-10 for the counters (block, step, ant, iter) of one ant's step,
// where only `block` differs between the candidates.  Rounds 0 and 1 multiply
// the ant word and the step's word 0 by the same constants for every
// candidate, so those products are taken once: per ant (PhiloxAnt, for the
// whole tour) and per step (PhiloxStep, for every batch of the step).  What
// remains per candidate is one multiply in rounds 0 and 1, two from round 2
// on, and a two- or three-input XOR per new word.  The outputs are the same
// four words as philox10_block's.
struct PhiloxAnt {
    uint32_t h;   // hi(ant * kMulB) ^ k0: word 0 after round 0 is h ^ step
    uint32_t u1;  // lo(ant * kMulB): word 1 after round 0
};

struct PhiloxStep {
    uint32_t u1;   // word 1 after round 0 (the ant's)
    uint32_t v1;   // hi(word 0 after round 0 * kMulA) ^ round-1 key 1: word 2 after round 1 is word 3 ^ v1
    uint32_t v2;   // lo(word 0 after round 0 * kMulA) ^ round-2 key 1, folded into word 2 after round 2
};

constexpr uint32_t kPhiloxMulA = 0xD2511F53u;
constexpr uint32_t kPhiloxMulB = 0xCD9E8D57u;
constexpr uint32_t kPhiloxBumpA = 0x9E3779B9u;
constexpr uint32_t kPhiloxBumpB = 0xBB67AE85u;

__device__ __forceinline__ PhiloxAnt philox_ant(uint32_t ant, uint32_t k0) {
    const uint64_t pb = static_cast<uint64_t>(ant) * kPhiloxMulB;
    return PhiloxAnt{static_cast<uint32_t>(pb >> 32) ^ k0, static_cast<uint32_t>(pb)};
}

__device__ __forceinline__ PhiloxStep philox_step(const PhiloxAnt& a, uint32_t step,
                                                  uint32_t k1) {
    const uint64_t pa = static_cast<uint64_t>(a.h ^ step) * kPhiloxMulA;
    return PhiloxStep{a.u1, static_cast<uint32_t>(pa >> 32) ^ (k1 + kPhiloxBumpB),
                      static_cast<uint32_t>(pa) ^ (k1 + 2u * kPhiloxBumpB)};
}

// `iter_k1` is iter ^ k1 (wave-uniform).
__device__ __forceinline__ PhiloxOut philox10_candidate(uint32_t block, const PhiloxStep& st,
                                                       uint32_t iter_k1, uint32_t k0,
                                                       uint32_t k1) {
    // round 0: word 0 and word 1 come from the ant and the step
    const uint64_t pa0 = static_cast<uint64_t>(block) * kPhiloxMulA;
    const uint32_t x2a = static_cast<uint32_t>(pa0 >> 32) ^ iter_k1;
    const uint32_t x3a = static_cast<uint32_t>(pa0);
    // round 1: word 0's product is the step's
    const uint64_t pb1 = static_cast<uint64_t>(x2a) * kPhiloxMulB;
    const uint32_t x0b = xor3_vvs(static_cast<uint32_t>(pb1 >> 32), st.u1, k0 + kPhiloxBumpA);
    const uint32_t x1b = static_cast<uint32_t>(pb1);
    const uint32_t x2b = x3a ^ st.v1;
    // round 2: word 3 after round 1 is the step's
    const uint64_t pa2 = static_cast<uint64_t>(x0b) * kPhiloxMulA;
    const uint64_t pb2 = static_cast<uint64_t>(x2b) * kPhiloxMulB;
    uint32_t x0 = xor3_vvs(static_cast<uint32_t>(pb2 >> 32), x1b, k0 + 2u * kPhiloxBumpA);
    uint32_t x1 = static_cast<uint32_t>(pb2);
    uint32_t x2 = static_cast<uint32_t>(pa2 >> 32) ^ st.v2;
    uint32_t x3 = static_cast<uint32_t>(pa2);
#pragma unroll
    for (int r = 3; r < 10; ++r) {
        const uint64_t pa = static_cast<uint64_t>(x0) * kPhiloxMulA;
        const uint64_t pb = static_cast<uint64_t>(x2) * kPhiloxMulB;
        const uint32_t n0 = xor3_vvs(static_cast<uint32_t>(pb >> 32), x1,
                                     k0 + static_cast<uint32_t>(r) * kPhiloxBumpA);
        const uint32_t n2 = xor3_vvs(static_cast<uint32_t>(pa >> 32), x3,
                                     k1 + static_cast<uint32_t>(r) * kPhiloxBumpB);
        x0 = n0;
        x1 = static_cast<uint32_t>(pb);
        x2 = n2;
        x3 = static_cast<uint32_t>(pa);
    }
    return PhiloxOut{x0, x1, x2, x3};
}

// (2*(w >> 9) + 1) * 2^-24 without a conversion: OR the top 23 bits into the
// mantissa of 1.0f, giving 1 + k*2^-23 in [1, 2), then subtract 1 - 2^-24.
// The difference (2k+1)*2^-24 has at most 24 significant bits, so the FP32
// subtraction is exact.
__device__ __forceinline__ float unit_from_word(uint32_t w) {
    return __uint_as_float(0x3F800000u | (w >> 9)) - 0x1.fffffep-1f;
}

}  // namespace aco
