// storage.hpp -- encodings of the stored population deviations (FP32, FP16, BF16)
// and the AA-pattern slot of population i at node x.
//
// The stored value is q = (f_i - w_i rho0) / sigma_class(i); sigma is 1 for FP32
// and the thermal scale sqrt(w_i rho0 kT / cs^2) (or a user scale) for 16-bit
// storage, so thermal noise is O(1) in storage units.  Stores round to nearest
// even.
#pragma once
#include <cstdint>
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace rflbm {

template <int S>
struct Codec;

// decode(q, sigma) = q sigma; decode_add(q, sigma, c) = q sigma + c and
// decode_sub(q, sigma, c) = c - q sigma, each one rounding (a fused
// multiply-add, or an exact add where sigma is 1).
template <>
struct Codec<kF32> {
  using T = float;
  __device__ __forceinline__ static float decode(T q, float) { return q; }
  __device__ __forceinline__ static float decode_add(T q, float, float c) { return q + c; }
  __device__ __forceinline__ static float decode_sub(T q, float, float c) { return c - q; }
  __device__ __forceinline__ static T encode(float d, float) { return d; }
};

template <>
struct Codec<kF16> {
  using T = _Float16;
  __device__ __forceinline__ static float decode(T q, float sigma) {
    return static_cast<float>(q) * sigma;
  }
  __device__ __forceinline__ static float decode_add(T q, float sigma, float c) {
    return fmaf(static_cast<float>(q), sigma, c);
  }
  __device__ __forceinline__ static float decode_sub(T q, float sigma, float c) {
    return fmaf(static_cast<float>(q), -sigma, c);
  }
  __device__ __forceinline__ static T encode(float d, float inv_sigma) {
    return static_cast<_Float16>(d * inv_sigma);
  }
};

template <>
struct Codec<kBF16> {
  using T = uint16_t;  // raw bfloat16 bits
  __device__ __forceinline__ static float widen(T q) { return __uint_as_float(static_cast<uint32_t>(q) << 16); }
  __device__ __forceinline__ static float decode(T q, float sigma) { return widen(q) * sigma; }
  __device__ __forceinline__ static float decode_add(T q, float sigma, float c) { return fmaf(widen(q), sigma, c); }
  __device__ __forceinline__ static float decode_sub(T q, float sigma, float c) { return fmaf(widen(q), -sigma, c); }
  __device__ __forceinline__ static T encode(float d, float inv_sigma) {
    const uint32_t u = __float_as_uint(d * inv_sigma);
    // round to nearest even on the 16 dropped bits (finite inputs)
    return static_cast<T>((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
  }
};

// Byte size of one stored value.
constexpr int storage_bytes(int s) { return s == kF32 ? 4 : 2; }

// A stored element as a 32-bit word (16-bit types zero-extended) and back.
template <class T>
__device__ __forceinline__ uint32_t to_bits(T q) {
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(uint32_t, q);
  else return __builtin_bit_cast(uint16_t, q);
}
template <class T>
__device__ __forceinline__ T from_bits(uint32_t b) {
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, b);
  else return __builtin_bit_cast(T, static_cast<uint16_t>(b));
}

// Periodic neighbour coordinate: c in {-1, 0, 1}.
__host__ __device__ __forceinline__ uint32_t wrap_add(uint32_t x, int c, uint32_t n) {
  return c == 0 ? x : (c > 0 ? (x + 1 == n ? 0u : x + 1) : (x == 0 ? n - 1 : x - 1));
}

}  // namespace rflbm
