// fastdiv.hpp -- unsigned 32-bit division by a run-time constant d >= 2 with
// one high multiply (Granlund and Montgomery, "Division by invariant integers
// using multiplication", PLDI 1994, the round-up variant with a 33-bit
// multiplier split as m + 2^32):
//   s = ceil(log2 d),  m = floor(2^32 (2^s - d) / d) + 1,
//   q = (t + ((n - t) >> 1)) >> (s - 1),  t = floor(m n / 2^32),
// exact for every n < 2^32.  Used to turn a flattened node index into (x, y, z)
// in the batched kernel, and block indices into tile or row coordinates in the
// one-box kernels (there the operands are uniform, so the divisions stay on the
// scalar unit).  Host-only code may include this header without HIP.
#pragma once
#include <cstdint>

namespace rflbm {

struct FastDiv {
  uint32_t m;  // magic multiplier
  uint32_t s;  // ceil(log2 d), >= 1
};

inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t s = 0;
  while ((uint64_t(1) << s) < d) ++s;
  const uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << s) - d)) / d + 1;
  return FastDiv{static_cast<uint32_t>(m), s};
}

#if defined(__HIPCC__)
#define RFLBM_HD __host__ __device__
#else
#define RFLBM_HD
#endif

RFLBM_HD inline uint32_t fast_div(uint32_t n, FastDiv f) {
#if defined(__HIP_DEVICE_COMPILE__)
  const uint32_t t = __umulhi(n, f.m);
#else
  const uint32_t t = static_cast<uint32_t>((static_cast<uint64_t>(n) * f.m) >> 32);
#endif
  return (t + ((n - t) >> 1)) >> (f.s - 1);
}

// n / d for any d >= 1 (make_fastdiv needs d >= 2; d = 1 is the identity).
RFLBM_HD inline uint32_t div_by(uint32_t n, uint32_t d, FastDiv f) { return d == 1 ? n : fast_div(n, f); }

}  // namespace rflbm
