// philox.hpp -- counter-based normal random numbers for the noise term of the
// fluctuating update (arXiv:2507.08820, Eq. fluct_phi: r_k ~ N(0, 1); the paper
// does not name its generator).
//
// Generator: Philox4x32 of Salmon, Moraes, Dror and Shaw, "Parallel random
// numbers: as easy as 1, 2, 3" (SC'11).  One round takes the 128-bit counter as
// four 32-bit words, forms the 64-bit products of words 0 and 2 with two fixed
// odd multipliers, and returns (hi(product 2) ^ word 1 ^ key 0,
// lo(product 2), hi(product 0) ^ word 3 ^ key 1, lo(product 0)); the two key
// words advance by Weyl increments between rounds.
//
// Use in the step kernel: key = (seed low, seed high), counter =
// (node, step, call j, stream id), j = 0..5.  Words (0, 1) and (2, 3) of a call
// are Box-Muller pairs, each word giving a uniform from its top 23 bits
// b = w >> 9: the radius word U0 = 1 - b 2^-23 in [2^-23, 1], the angle word
// U1 = b 2^-23 in [0, 1); R = sqrt(-2 ln U0), z0 = R cos(2 pi U1),
// z1 = R sin(2 pi U1).  Both are read off one float: the bits 0x3F800000 | b
// are X = 1 + b 2^-23 in [1, 2), so U0 = 2 - X (exact) and, since the gfx950
// sine and cosine take their argument in revolutions and are periodic in it,
// cos(2 pi U1) is the hardware cosine of X itself.  The hardware logarithm is
// base 2, so ln U0 = ln 2 log2 U0.
#pragma once
#include <cstdint>
#include <hip/hip_runtime.h>

namespace rflbm {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;  // multiplier of word 0
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;  // multiplier of word 2
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;  // key-0 increment (golden ratio)
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;  // key-1 increment (sqrt(3) - 1)

struct Word4 {
  uint32_t w0, w1, w2, w3;
};

// a ^ b ^ c: one gfx950 three-input bitwise instruction (truth table 0x96)
// instead of two exclusive-ors.
__host__ __device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
  return a ^ b ^ c;
#endif
}

// R rounds of Philox4x32 on counter c with key (k0, k1).
template <int R>
__host__ __device__ __forceinline__ Word4 philox(Word4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint64_t p0 = static_cast<uint64_t>(kPhiloxM0) * c.w0;
    const uint64_t p2 = static_cast<uint64_t>(kPhiloxM1) * c.w2;
    Word4 n;
    n.w0 = xor3(static_cast<uint32_t>(p2 >> 32), c.w1, k0);
    n.w1 = static_cast<uint32_t>(p2);
    n.w2 = xor3(static_cast<uint32_t>(p0 >> 32), c.w3, k1);
    n.w3 = static_cast<uint32_t>(p0);
    c = n;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return c;
}

// X = 1 + (w >> 9) 2^-23 in [1, 2): the top 23 bits of w as the mantissa of a
// float of exponent 0 (one bit-field instruction).
__device__ __forceinline__ float word_to_one_two(uint32_t w) {
  return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, w, 9));
}

// The radius uniform 1 - (w >> 9) 2^-23 in [2^-23, 1] and the angle uniform
// (w >> 9) 2^-23 in [0, 1) of a word, exact in FP32.
__device__ __forceinline__ float radius_uniform(uint32_t w) { return 2.0f - word_to_one_two(w); }
__device__ __forceinline__ float angle_uniform(uint32_t w) { return word_to_one_two(w) - 1.0f; }

constexpr float kMinus2Ln2 = -1.38629436111989061883f;  // -2 ln 2

// Box-Muller pair from two words (radius word, angle word), both normals
// multiplied by sqrt(c / (-2 ln 2)): the radius is sqrt(c log2 U0), so c = -2 ln 2
// gives standard normals and c = -2 ln 2 rho gives sqrt(rho) times them.
__device__ __forceinline__ void box_muller_scaled(uint32_t wr, uint32_t wa, float c, float& z0, float& z1) {
  const float ur = radius_uniform(wr);
  const float turns = word_to_one_two(wa);  // 1 + the angle uniform, in revolutions
  const float rad = __builtin_amdgcn_sqrtf(c * __builtin_amdgcn_logf(ur));
  z0 = rad * __builtin_amdgcn_cosf(turns);
  z1 = rad * __builtin_amdgcn_sinf(turns);
}

// Standard normal Box-Muller pair.
__device__ __forceinline__ void box_muller(uint32_t wr, uint32_t wa, float& z0, float& z1) {
  box_muller_scaled(wr, wa, kMinus2Ln2, z0, z1);
}

}  // namespace rflbm
