// d3q27.hpp -- D3Q27 lattice constants and separable Hermite transforms for the
// GPU path (arXiv:2507.08820, Sec. II: Table I velocities and weights, Table II
// Hermite basis).
//
// Every Table II polynomial is a product over the three axes of a 1-D
// polynomial of degree p in {0, 1, 2}: 1, c, c^2 - cs^2 (cs^2 = 1/3).  Mode k
// therefore has a degree triple (px, py, pz), its norm is
// b_k = beta(px) beta(py) beta(pz) with beta = (1, 1/3, 2/9), and the weights
// factor as w_i = omega(cx) omega(cy) omega(cz) with omega(0) = 2/3,
// omega(+-1) = 1/6.  The 27x27 projection m_k = sum_i e_ki f_i (Eq. moments)
// and its inverse f_i = w_i sum_k b_k^-1 e_ki m_k (Eq. backtrasf) thus split
// into three sweeps of a 3-point transform along x, y and z.
//
// Register layout used by the kernels: population i = ix + 3 iy + 9 iz with
// i_a = c_a + 1; after the forward sweeps, slot px + 3 py + 9 pz holds the
// moment of degrees (px, py, pz).
#pragma once
#include <cstdint>

namespace rflbm {

constexpr int kQ = 27;

// Degree triple (px, py, pz) of Table II mode k, k = 0..26 in the table's order.
constexpr int kModeDeg[kQ][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1},                       // H0, Hx, Hy, Hz
    {2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, // second order
    {2, 1, 0}, {2, 0, 1}, {1, 2, 0}, {1, 0, 2}, {0, 1, 2}, {0, 2, 1}, {1, 1, 1},  // third
    {2, 2, 0}, {2, 0, 2}, {0, 2, 2}, {1, 1, 2}, {1, 2, 1}, {2, 1, 1},  // fourth
    {2, 1, 2}, {2, 2, 1}, {1, 2, 2},                                   // fifth
    {2, 2, 2}};                                                        // sixth

// Register slot of Table II mode k.
constexpr int mode_slot(int k) { return kModeDeg[k][0] + 3 * kModeDeg[k][1] + 9 * kModeDeg[k][2]; }

// Weight class |c_i|^2 of population i (0: rest, 1: axis, 2: face, 3: corner).
constexpr int speed_class(int i) {
  return (i % 3 != 1) + ((i / 3) % 3 != 1) + (i / 9 != 1);
}

// Weights w_i = (2/3)^(3 - class) (1/6)^class, in double for host set-up.
constexpr double class_weight(int cls) {
  return cls == 0 ? 8.0 / 27.0 : cls == 1 ? 2.0 / 27.0 : cls == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
}

// Hermite norm b_k = prod_a beta(p_a), beta = (1, 1/3, 2/9).
constexpr double mode_norm(int k) {
  double b = 1.0;
  for (int a = 0; a < 3; ++a) b *= kModeDeg[k][a] == 0 ? 1.0 : kModeDeg[k][a] == 1 ? 1.0 / 3.0 : 2.0 / 9.0;
  return b;
}

// Forward 3-point transform along one axis: (f-, f0, f+) -> degrees (0, 1, 2):
// sum f, f+ - f-, sum (c^2 - 1/3) f = (f- + f+) - (sum f) / 3.
__host__ __device__ __forceinline__ void fwd3(float& lo, float& mid, float& hi) {
  const float s = lo + hi;
  const float d = hi - lo;
  const float m0 = s + mid;
  lo = m0;
  mid = d;
  hi = fmaf(-1.0f / 3.0f, m0, s);
}

// Inverse 3-point transform: degrees (m0, m1, m2) -> (f-, f0, f+) with
// f_c = omega(c) sum_p beta(p)^-1 P_p(c) m_p:
// f0 = 2/3 m0 - m2,  f+- = 1/6 m0 + 1/2 m2 +- 1/2 m1.
__host__ __device__ __forceinline__ void inv3(float& lo, float& mid, float& hi) {
  const float m0 = lo, m1 = mid, m2 = hi;
  const float t = 0.5f * fmaf(1.0f / 3.0f, m0, m2);
  const float h = 0.5f * m1;
  lo = t - h;
  hi = t + h;
  mid = fmaf(2.0f / 3.0f, m0, -m2);
}

// Scaled inverse.  With the degree-p input of a 3-point inverse pre-multiplied by
// s(p), s = (2/3, 1/2, 1/2), the transform takes four operations:
// f0 = m0' - 2 m2', f+- = m0' / 4 + m2' +- m1'.  Pre-multiplying mode
// (px, py, pz) by inv_scale = s(px) s(py) s(pz) lets all three sweeps use it,
// since each sweep is linear and leaves the other axes' factors in place.
constexpr double inv_axis_scale(int p) { return p == 0 ? 2.0 / 3.0 : 0.5; }
constexpr double inv_scale(int slot) {
  return inv_axis_scale(slot % 3) * inv_axis_scale((slot / 3) % 3) * inv_axis_scale(slot / 9);
}

__host__ __device__ __forceinline__ void inv3_scaled(float& lo, float& mid, float& hi) {
  const float m0 = lo, m1 = mid, m2 = hi;
  const float t = fmaf(0.25f, m0, m2);
  lo = t - m1;
  hi = t + m1;
  mid = fmaf(-2.0f, m2, m0);
}

// The y and z sweeps of the forward transform (after the x sweep).
__host__ __device__ __forceinline__ void forward27_yz(float v[kQ]) {
#pragma unroll
  for (int iz = 0; iz < 3; ++iz)
#pragma unroll
    for (int ix = 0; ix < 3; ++ix) fwd3(v[ix + 9 * iz], v[ix + 3 + 9 * iz], v[ix + 6 + 9 * iz]);  // y
#pragma unroll
  for (int g = 0; g < 9; ++g) fwd3(v[g], v[g + 9], v[g + 18]);  // z
}

// In-place forward transform of the 27 registers: populations -> moments.
__host__ __device__ __forceinline__ void forward27(float v[kQ]) {
#pragma unroll
  for (int g = 0; g < 9; ++g) fwd3(v[3 * g], v[3 * g + 1], v[3 * g + 2]);  // x
  forward27_yz(v);
}

// In-place inverse transform: moments -> populations.
__host__ __device__ __forceinline__ void inverse27(float v[kQ]) {
#pragma unroll
  for (int g = 0; g < 9; ++g) inv3(v[g], v[g + 9], v[g + 18]);  // z
#pragma unroll
  for (int iz = 0; iz < 3; ++iz)
#pragma unroll
    for (int ix = 0; ix < 3; ++ix) inv3(v[ix + 9 * iz], v[ix + 3 + 9 * iz], v[ix + 6 + 9 * iz]);  // y
#pragma unroll
  for (int g = 0; g < 9; ++g) inv3(v[3 * g], v[3 * g + 1], v[3 * g + 2]);  // x
}

// In-place inverse of pre-scaled moments (slot s holding inv_scale(s) m):
// moments -> populations, the same result as inverse27 on unscaled moments.
__host__ __device__ __forceinline__ void inverse27_scaled(float v[kQ]) {
#pragma unroll
  for (int g = 0; g < 9; ++g) inv3_scaled(v[g], v[g + 9], v[g + 18]);  // z
#pragma unroll
  for (int iz = 0; iz < 3; ++iz)
#pragma unroll
    for (int ix = 0; ix < 3; ++ix) inv3_scaled(v[ix + 9 * iz], v[ix + 3 + 9 * iz], v[ix + 6 + 9 * iz]);  // y
#pragma unroll
  for (int g = 0; g < 9; ++g) inv3_scaled(v[3 * g], v[3 * g + 1], v[3 * g + 2]);  // x
}

}  // namespace rflbm
