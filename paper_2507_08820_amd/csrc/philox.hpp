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
// (node, step, call j, stream id), j = 0..3.  The four words of a call carry
// three Box-Muller pairs m = 0, 1, 2: the radius of pair m from the top 23
// bits b = w_m >> 9 of word m, U0 = 1 - b 2^-23 in [2^-23, 1]; its angle from
// 16 bits a no radius uses, U1 = a 2^-16 in [0, 1): a = w3 >> 16, w3 & 0xFFFF,
// and (w0 & 0xFF) 2^8 + (w1 & 0xFF) for m = 0, 1, 2.  R = sqrt(-2 ln U0),
// z0 = R cos(2 pi U1), z1 = R sin(2 pi U1).  Both uniforms are read off
// floats in [1, 2): the bits 0x3F800000 | b are X = 1 + b 2^-23, so
// U0 = 2 - X (exact), and the bits 0x3F800000 | a 2^7 are 1 + U1; since the
// gfx950 sine and cosine take their argument in revolutions and are periodic
// in it, cos(2 pi U1) is the hardware cosine of 1 + U1 itself.  The hardware
// logarithm is base 2, so ln U0 = ln 2 log2 U0.
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

// The radius uniform 1 - (w >> 9) 2^-23 in [2^-23, 1] of a word, exact in FP32.
__device__ __forceinline__ float radius_uniform(uint32_t w) { return 2.0f - word_to_one_two(w); }

// 1 + a 2^-16 in [1, 2) for the 16 angle bits a of pair m of a call: the
// 16-bit field placed at the top of the mantissa of a float of exponent 0.
template <int M>
__device__ __forceinline__ float angle_one_two(const Word4& w) {
  uint32_t mant;
  if constexpr (M == 0) mant = (w.w3 >> 9) & 0x7FFF80u;         // a = w3 >> 16
  else if constexpr (M == 1) mant = (w.w3 << 7) & 0x7FFF80u;    // a = w3 & 0xFFFF
  else mant = ((w.w0 & 0xFFu) << 15) | ((w.w1 & 0xFFu) << 7);   // a = (w0 & 0xFF) 2^8 + (w1 & 0xFF)
  return __uint_as_float(0x3F800000u | mant);
}

// The angle uniform a 2^-16 in [0, 1) of pair m, exact in FP32.
template <int M>
__device__ __forceinline__ float angle_uniform(const Word4& w) { return angle_one_two<M>(w) - 1.0f; }

constexpr float kMinus2Ln2 = -1.38629436111989061883f;  // -2 ln 2

// Box-Muller pair m of a call, both normals multiplied by sqrt(c / (-2 ln 2)):
// the radius is sqrt(c log2 U0), so c = -2 ln 2 gives standard normals and
// c = -2 ln 2 rho gives sqrt(rho) times them.
template <int M>
__device__ __forceinline__ void box_muller_scaled(const Word4& w, float c, float& z0, float& z1) {
  const uint32_t wr = M == 0 ? w.w0 : (M == 1 ? w.w1 : w.w2);
  const float ur = radius_uniform(wr);
  const float turns = angle_one_two<M>(w);  // 1 + the angle uniform, in revolutions
  const float rad = __builtin_amdgcn_sqrtf(c * __builtin_amdgcn_logf(ur));
  z0 = rad * __builtin_amdgcn_cosf(turns);
  z1 = rad * __builtin_amdgcn_sinf(turns);
}

// Standard normal Box-Muller pair m of a call.
template <int M>
__device__ __forceinline__ void box_muller(const Word4& w, float& z0, float& z1) {
  box_muller_scaled<M>(w, kMinus2Ln2, z0, z1);
}

}  // namespace rflbm
