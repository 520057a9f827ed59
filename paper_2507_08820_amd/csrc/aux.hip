// aux.hip -- kernels around the step: population readback and write-back in the
// canonical FP64 layout, equilibrium initialisation (Eq. hermite_feq2 in its
// product form), moment fields rho, j, Pi (Eqs. eq:rho, eq:u and the Pi of
// Sec. III), re-encoding of stored deviations, the noise generator exposed for
// testing, and a plain copy kernel (bandwidth reference).
//
// All of these work on the AA layout described in kernels.hpp: at an even step
// count f_i(x) sits in slot A[i][x], at an odd one in A[26 - i][x - c_i].
#include <hip/hip_runtime.h>

#include "d3q27.hpp"
#include "kernels.hpp"
#include "philox.hpp"
#include "storage.hpp"

namespace rflbm {

namespace {

struct NodeXYZ {
  uint32_t x, y, z;
};

__device__ __forceinline__ NodeXYZ coords(uint64_t n, uint32_t nx, uint32_t ny) {
  NodeXYZ c;
  c.x = static_cast<uint32_t>(n % nx);
  const uint64_t r = n / nx;
  c.y = static_cast<uint32_t>(r % ny);
  c.z = static_cast<uint32_t>(r / ny);
  return c;
}

// Element index of slot A[plane][(x, y, z)] in the x-row blocked layout, its
// row blocks in By x Bz bricks (kernels.hpp; By = Bz = 1: plain layout).
__device__ __forceinline__ uint64_t element_index(int plane, uint32_t x, uint32_t y, uint32_t z,
                                                  const GatherArgs& g) {
  const uint64_t yo = (y >> g.by_log) * g.ybrick_pitch + (y & ((1u << g.by_log) - 1u)) * g.row_pitch;
  const uint64_t zo = (z >> g.bz_log) * g.plane_pitch + (z & ((1u << g.bz_log) - 1u)) * g.zin_pitch;
  return zo + yo + static_cast<uint64_t>(plane) * g.pop_pitch + x;
}

// Element index of the slot holding f_i(x) at the given parity.
__device__ __forceinline__ uint64_t slot_index(int i, NodeXYZ p, const GatherArgs& g) {
  if (!g.odd) return element_index(i, p.x, p.y, p.z, g);
  const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
  return element_index(kQ - 1 - i, wrap_add(p.x, -cx, g.nx), wrap_add(p.y, -cy, g.ny),
                       wrap_add(p.z, -cz, g.nz), g);
}

template <int S>
__global__ void get_pop_kernel(const GatherArgs g, double* dst) {
  using C = Codec<S>;
  using T = typename C::T;
  const uint64_t N = static_cast<uint64_t>(g.nx) * g.ny * g.nz;
  const T* pop = static_cast<const T*>(g.pop);
  for (uint64_t n = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; n < N;
       n += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const NodeXYZ p = coords(n, g.nx, g.ny);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int cls = speed_class(i);
      const float d = C::decode(pop[slot_index(i, p, g)], g.sigma[cls]);
      dst[i * N + n] = class_weight(cls) * g.rho0 + static_cast<double>(d);
    }
  }
}

template <int S>
__global__ void get_pop_at_kernel(const GatherArgs g, const uint32_t* nodes, uint32_t count, double* dst) {
  using C = Codec<S>;
  using T = typename C::T;
  const T* pop = static_cast<const T*>(g.pop);
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const uint32_t n = nodes[k];
  if (static_cast<uint64_t>(n) >= static_cast<uint64_t>(g.nx) * g.ny * g.nz) {
    // not a node of the box: nothing is read, the 27 values are NaN
#pragma unroll
    for (int i = 0; i < kQ; ++i) dst[static_cast<uint64_t>(i) * count + k] = __builtin_nan("");
    return;
  }
  const NodeXYZ p = coords(n, g.nx, g.ny);
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const int cls = speed_class(i);
    const float d = C::decode(pop[slot_index(i, p, g)], g.sigma[cls]);
    dst[static_cast<uint64_t>(i) * count + k] = class_weight(cls) * g.rho0 + static_cast<double>(d);
  }
}

template <int S>
__global__ void set_pop_kernel(const GatherArgs g, const double* src) {
  using C = Codec<S>;
  using T = typename C::T;
  const uint64_t N = static_cast<uint64_t>(g.nx) * g.ny * g.nz;
  T* pop = static_cast<T*>(const_cast<void*>(g.pop));
  for (uint64_t n = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; n < N;
       n += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const NodeXYZ p = coords(n, g.nx, g.ny);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int cls = speed_class(i);
      const double d = src[i * N + n] - class_weight(cls) * g.rho0;
      pop[slot_index(i, p, g)] = C::encode(static_cast<float>(d), g.inv_sigma[cls]);
    }
  }
}

// f^(0)_i = rho prod_a omega(c_a) [1 + c_a u_a / cs2 + (c_a^2 - cs2) u_a^2 / (2 cs2^2)],
// the product form of the full-Hermite equilibrium (every Table II mode is a
// product of 1-D Hermite polynomials, so its Hermite sum factorises by axis).
template <int S>
__global__ void init_eq_kernel(const GatherArgs g, const double* rho, const double* u) {
  using C = Codec<S>;
  using T = typename C::T;
  const uint64_t N = static_cast<uint64_t>(g.nx) * g.ny * g.nz;
  T* pop = static_cast<T*>(const_cast<void*>(g.pop));
  for (uint64_t n = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; n < N;
       n += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const NodeXYZ p = coords(n, g.nx, g.ny);
    const double r = rho ? rho[n] : g.rho0;
    const double ua[3] = {u ? u[n] : 0.0, u ? u[N + n] : 0.0, u ? u[2 * N + n] : 0.0};
    double fac[3][3];  // fac[a][c + 1]
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double q = 4.5 * ua[a] * ua[a];
      fac[a][0] = (1.0 / 6.0) * (1.0 - 3.0 * ua[a] + q - 1.5 * ua[a] * ua[a]);
      fac[a][1] = (2.0 / 3.0) * (1.0 - 1.5 * ua[a] * ua[a]);
      fac[a][2] = (1.0 / 6.0) * (1.0 + 3.0 * ua[a] + q - 1.5 * ua[a] * ua[a]);
    }
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int cls = speed_class(i);
      const double feq = r * fac[0][i % 3] * fac[1][(i / 3) % 3] * fac[2][i / 9];
      const double d = feq - class_weight(cls) * g.rho0;
      pop[slot_index(i, p, g)] = C::encode(static_cast<float>(d), g.inv_sigma[cls]);
    }
  }
}

// Thermalised start: f_i = f^(0)_i(rho, u) + sqrt(rho0 kT w_i / cs2) xi_i, the
// stationary covariance of the fluctuating update (Eq. fluct_phi) in the
// linear regime.  xi_i is normal i of the node's Box-Muller stream at the
// reserved step word 0xFFFFFFFF, Philox calls j = 0..4 (30 normals, 27 used);
// set-up code, so the transform runs in FP64.
template <int S, int R>
__global__ void init_thermal_kernel(const GatherArgs g, const double* rho, const double* u, uint32_t key0,
                                    uint32_t key1, uint32_t sid, double kT) {
  using C = Codec<S>;
  using T = typename C::T;
  const uint64_t N = static_cast<uint64_t>(g.nx) * g.ny * g.nz;
  T* pop = static_cast<T*>(const_cast<void*>(g.pop));
  const double mu = g.rho0 * kT * 3.0;
  for (uint64_t n = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; n < N;
       n += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const NodeXYZ p = coords(n, g.nx, g.ny);
    const double r = rho ? rho[n] : g.rho0;
    const double ua[3] = {u ? u[n] : 0.0, u ? u[N + n] : 0.0, u ? u[2 * N + n] : 0.0};
    double fac[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double uu = ua[a] * ua[a];
      fac[a][0] = (1.0 / 6.0) * (1.0 - 3.0 * ua[a] + 3.0 * uu);
      fac[a][1] = (2.0 / 3.0) * (1.0 - 1.5 * uu);
      fac[a][2] = (1.0 / 6.0) * (1.0 + 3.0 * ua[a] + 3.0 * uu);
    }
    double z[30];
#pragma unroll
    for (uint32_t j = 0; j < 5; ++j) {
      const Word4 w = philox<R>(Word4{static_cast<uint32_t>(n), 0xFFFFFFFFu, j, sid}, key0, key1);
      // pair m: radius uniform 1 - (w_m >> 9) 2^-23, angle uniform a_m 2^-16
      const uint32_t wr[3] = {w.w0, w.w1, w.w2};
      const uint32_t am[3] = {w.w3 >> 16, w.w3 & 0xFFFFu, ((w.w0 & 0xFFu) << 8) | (w.w1 & 0xFFu)};
      const double two_pi = 6.283185307179586476925;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const double ur = 1.0 - static_cast<double>(wr[m] >> 9) * 0x1p-23;
        const double ua = static_cast<double>(am[m]) * 0x1p-16;
        const double rad = sqrt(-2.0 * log(ur));
        z[6 * j + 2 * m] = rad * cos(two_pi * ua);
        z[6 * j + 2 * m + 1] = rad * sin(two_pi * ua);
      }
    }
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int cls = speed_class(i);
      const double w = class_weight(cls);
      const double feq = r * fac[0][i % 3] * fac[1][(i / 3) % 3] * fac[2][i / 9];
      const double d = feq - w * g.rho0 + sqrt(mu * w) * z[i];
      pop[slot_index(i, p, g)] = C::encode(static_cast<float>(d), g.inv_sigma[cls]);
    }
  }
}

// Moment fields of the nodes n0 .. n0 + count - 1: field c of node n0 + k goes
// to dst[c * pitch + k].
template <int S>
__global__ void moments_kernel(const GatherArgs g, uint32_t mask, uint64_t n0, uint64_t count,
                               uint64_t pitch, float* dst) {
  using C = Codec<S>;
  using T = typename C::T;
  const T* pop = static_cast<const T*>(g.pop);
  for (uint64_t k = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; k < count;
       k += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const NodeXYZ p = coords(n0 + k, g.nx, g.ny);
    float v[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) v[i] = C::decode(pop[slot_index(i, p, g)], g.sigma[speed_class(i)]);
    forward27(v);
    float* out = dst;
    if (mask & 1u) {
      out[k] = static_cast<float>(g.rho0 + static_cast<double>(v[0]));
      out += pitch;
    }
    if (mask & 2u) {
      out[k] = v[1];
      out[pitch + k] = v[3];
      out[2 * pitch + k] = v[9];
      out += 3 * pitch;
    }
    if (mask & 4u) {
      const int slots[6] = {mode_slot(4), mode_slot(5), mode_slot(6), mode_slot(7), mode_slot(8), mode_slot(9)};
#pragma unroll
      for (int c = 0; c < 6; ++c) out[c * pitch + k] = v[slots[c]];
    }
  }
}

// Slot A[p][.] holds populations of one speed class at either parity (26 - i
// and i have the same |c|^2), so re-encoding works slot by slot.
template <int S>
__global__ void reencode_kernel(const GatherArgs from, const GatherArgs to) {
  using C = Codec<S>;
  using T = typename C::T;
  const uint64_t N = static_cast<uint64_t>(from.nx) * from.ny * from.nz;
  T* pop = static_cast<T*>(const_cast<void*>(from.pop));
  const uint64_t total = N * kQ;
  for (uint64_t e = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    // e runs over (x, plane, y, z) with x fastest; padding is left untouched
    const uint32_t x = static_cast<uint32_t>(e % from.nx);
    const uint64_t r = e / from.nx;
    const int plane = static_cast<int>(r % kQ);
    const uint64_t row = r / kQ;
    const int cls = speed_class(plane);
    T* q = pop + element_index(plane, x, static_cast<uint32_t>(row % from.ny),
                               static_cast<uint32_t>(row / from.ny), from);
    const double d = static_cast<double>(C::decode(*q, from.sigma[cls])) +
                     class_weight(cls) * (from.rho0 - to.rho0);
    *q = C::encode(static_cast<float>(d), to.inv_sigma[cls]);
  }
}

template <int R>
__global__ void rng_kernel(uint32_t key0, uint32_t key1, uint32_t sid, uint32_t node0, uint32_t count,
                           uint32_t step, float* u, float* z) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const uint32_t node = node0 + t;
#pragma unroll
  for (uint32_t j = 0; j < 4; ++j) {
    const Word4 w = philox<R>(Word4{node, step, j, sid}, key0, key1);
    float r[6], uu[6];
    box_muller<0>(w, r[0], r[1]);
    box_muller<1>(w, r[2], r[3]);
    box_muller<2>(w, r[4], r[5]);
    uu[0] = radius_uniform(w.w0);
    uu[1] = angle_uniform<0>(w);
    uu[2] = radius_uniform(w.w1);
    uu[3] = angle_uniform<1>(w);
    uu[4] = radius_uniform(w.w2);
    uu[5] = angle_uniform<2>(w);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      u[static_cast<uint64_t>(t) * 24 + 6 * j + q] = uu[q];
      z[static_cast<uint64_t>(t) * 24 + 6 * j + q] = r[q];
    }
  }
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// One 16-byte vector per thread, non-temporal loads and stores: the fastest
// of the copy forms measured on MI355X (one to eight vectors per thread,
// with and without non-temporal hints).
__global__ void __launch_bounds__(256) copy_kernel(u32x4* __restrict__ dst, const u32x4* __restrict__ src,
                                                   uint64_t n) {
  const uint64_t e = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (e < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + e), dst + e);
}

__global__ void fill_zero_kernel(double* dst, uint64_t n) {
  for (uint64_t e = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    dst[e] = 0.0;
}

__global__ void set_u32_kernel(uint32_t* dst, uint32_t value) {
  if (threadIdx.x == 0) *dst = value;
}

// Parity change of the stored state: the slot of f_j(y) at the new parity is
// A'[j][y] = A[26 - j][y - c_j] of the old one, in either direction.  The three
// kernels below move raw stored words (W = the storage word) so that the state
// is carried over bit for bit.
// tmp[n] = A[plane][n] (tmp compact, node order).
template <typename W>
__global__ void plane_save_kernel(const GatherArgs g, int plane, W* tmp) {
  const W* pop = static_cast<const W*>(g.pop);
  const uint64_t N = static_cast<uint64_t>(g.nx) * g.ny * g.nz;
  for (uint64_t n = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; n < N;
       n += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const NodeXYZ p = coords(n, g.nx, g.ny);
    tmp[n] = pop[element_index(plane, p.x, p.y, p.z, g)];
  }
}

// A[dst][y] = A[src][y - c] (dst != src), periodic.
template <typename W>
__global__ void plane_shift_kernel(const GatherArgs g, int dst, int src, int cx, int cy, int cz) {
  W* pop = static_cast<W*>(const_cast<void*>(g.pop));
  const uint64_t N = static_cast<uint64_t>(g.nx) * g.ny * g.nz;
  for (uint64_t n = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; n < N;
       n += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const NodeXYZ p = coords(n, g.nx, g.ny);
    pop[element_index(dst, p.x, p.y, p.z, g)] =
        pop[element_index(src, wrap_add(p.x, -cx, g.nx), wrap_add(p.y, -cy, g.ny), wrap_add(p.z, -cz, g.nz), g)];
  }
}

// A[dst][y] = tmp[y - c], periodic.
template <typename W>
__global__ void plane_restore_kernel(const GatherArgs g, int dst, const W* tmp, int cx, int cy, int cz) {
  W* pop = static_cast<W*>(const_cast<void*>(g.pop));
  const uint64_t N = static_cast<uint64_t>(g.nx) * g.ny * g.nz;
  for (uint64_t n = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; n < N;
       n += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const NodeXYZ p = coords(n, g.nx, g.ny);
    const uint64_t q = wrap_add(p.x, -cx, g.nx) +
                       static_cast<uint64_t>(g.nx) * (wrap_add(p.y, -cy, g.ny) +
                                                      static_cast<uint64_t>(g.ny) * wrap_add(p.z, -cz, g.nz));
    pop[element_index(dst, p.x, p.y, p.z, g)] = tmp[q];
  }
}


uint32_t grid_for(uint64_t work, uint32_t block) {
  const uint64_t g = (work + block - 1) / block;
  return static_cast<uint32_t>(g < 65536 ? (g == 0 ? 1 : g) : 65536);
}

template <typename W>
hipError_t swap_parity_words(const GatherArgs& g, W* tmp, hipStream_t s) {
  const uint64_t N = static_cast<uint64_t>(g.nx) * g.ny * g.nz;
  const dim3 grid(grid_for(N, 256)), block(256);
  // pairs (j, 26 - j), j < 13; the rest population (j = 13, c = 0) stays
  for (int j = 0; j < kQ / 2; ++j) {
    const int cx = j % 3 - 1, cy = (j / 3) % 3 - 1, cz = j / 9 - 1;
    hipLaunchKernelGGL(plane_save_kernel<W>, grid, block, 0, s, g, j, tmp);
    hipLaunchKernelGGL(plane_shift_kernel<W>, grid, block, 0, s, g, j, kQ - 1 - j, cx, cy, cz);
    hipLaunchKernelGGL(plane_restore_kernel<W>, grid, block, 0, s, g, kQ - 1 - j, tmp, -cx, -cy, -cz);
    if (const hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

#define RFLBM_DISPATCH_STORAGE(storage, KERNEL, grid, block, stream, ...)                  \
  do {                                                                                      \
    switch (storage) {                                                                      \
      case kF32: hipLaunchKernelGGL(KERNEL<kF32>, grid, block, 0, stream, __VA_ARGS__); break;   \
      case kF16: hipLaunchKernelGGL(KERNEL<kF16>, grid, block, 0, stream, __VA_ARGS__); break;   \
      case kBF16: hipLaunchKernelGGL(KERNEL<kBF16>, grid, block, 0, stream, __VA_ARGS__); break; \
      default: return hipErrorInvalidValue;                                                 \
    }                                                                                       \
  } while (0)

hipError_t launch_get_populations(int storage, const GatherArgs& g, double* dst, hipStream_t s) {
  const uint64_t N = static_cast<uint64_t>(g.nx) * g.ny * g.nz;
  RFLBM_DISPATCH_STORAGE(storage, get_pop_kernel, dim3(grid_for(N, 256)), dim3(256), s, g, dst);
  return hipGetLastError();
}

hipError_t launch_get_populations_at(int storage, const GatherArgs& g, const uint32_t* nodes, uint32_t count,
                                     double* dst, hipStream_t s) {
  if (count == 0) return hipSuccess;
  RFLBM_DISPATCH_STORAGE(storage, get_pop_at_kernel, dim3((count + 255) / 256), dim3(256), s, g, nodes, count, dst);
  return hipGetLastError();
}

hipError_t launch_set_populations(int storage, const GatherArgs& g, const double* src, hipStream_t s) {
  const uint64_t N = static_cast<uint64_t>(g.nx) * g.ny * g.nz;
  RFLBM_DISPATCH_STORAGE(storage, set_pop_kernel, dim3(grid_for(N, 256)), dim3(256), s, g, src);
  return hipGetLastError();
}

hipError_t launch_init_equilibrium(int storage, const GatherArgs& g, const double* rho,
                                   const double* u, hipStream_t s) {
  const uint64_t N = static_cast<uint64_t>(g.nx) * g.ny * g.nz;
  RFLBM_DISPATCH_STORAGE(storage, init_eq_kernel, dim3(grid_for(N, 256)), dim3(256), s, g, rho, u);
  return hipGetLastError();
}

hipError_t launch_init_thermal(int storage, const GatherArgs& g, const double* rho, const double* u,
                               uint32_t key0, uint32_t key1, uint32_t sid, int rounds, double kT,
                               hipStream_t s) {
  const uint64_t N = static_cast<uint64_t>(g.nx) * g.ny * g.nz;
  const dim3 grid(grid_for(N, 256)), block(256);
#define RFLBM_THERMAL(R)                                                                             \
  switch (storage) {                                                                                 \
    case kF32: hipLaunchKernelGGL((init_thermal_kernel<kF32, R>), grid, block, 0, s, g, rho, u, key0, key1, sid, kT); break;   \
    case kF16: hipLaunchKernelGGL((init_thermal_kernel<kF16, R>), grid, block, 0, s, g, rho, u, key0, key1, sid, kT); break;   \
    case kBF16: hipLaunchKernelGGL((init_thermal_kernel<kBF16, R>), grid, block, 0, s, g, rho, u, key0, key1, sid, kT); break; \
    default: return hipErrorInvalidValue;                                                            \
  }
  if (rounds == 10) {
    RFLBM_THERMAL(10)
  } else if (rounds == 7) {
    RFLBM_THERMAL(7)
  } else {
    return hipErrorInvalidValue;
  }
#undef RFLBM_THERMAL
  return hipGetLastError();
}

hipError_t launch_get_moments(int storage, const GatherArgs& g, uint32_t mask, float* dst,
                              hipStream_t s) {
  const uint64_t N = static_cast<uint64_t>(g.nx) * g.ny * g.nz;
  return launch_get_moments_range(storage, g, mask, 0, N, dst, N, s);
}

hipError_t launch_get_moments_range(int storage, const GatherArgs& g, uint32_t mask, uint64_t n0,
                                    uint64_t count, float* dst, uint64_t pitch, hipStream_t s) {
  if (count == 0) return hipSuccess;
  RFLBM_DISPATCH_STORAGE(storage, moments_kernel, dim3(grid_for(count, 256)), dim3(256), s, g, mask, n0,
                         count, pitch, dst);
  return hipGetLastError();
}

hipError_t launch_reencode(int storage, const GatherArgs& from, const GatherArgs& to, hipStream_t s) {
  const uint64_t N = static_cast<uint64_t>(from.nx) * from.ny * from.nz;
  RFLBM_DISPATCH_STORAGE(storage, reencode_kernel, dim3(grid_for(N * kQ, 256)), dim3(256), s, from, to);
  return hipGetLastError();
}

hipError_t launch_rng_normals(uint32_t key0, uint32_t key1, uint32_t stream_id, int rounds,
                              uint32_t node0, uint32_t count, uint32_t step, float* u, float* z,
                              hipStream_t s) {
  const dim3 grid((count + 255) / 256), block(256);
  if (count == 0) return hipSuccess;
  if (rounds == 10)
    hipLaunchKernelGGL(rng_kernel<10>, grid, block, 0, s, key0, key1, stream_id, node0, count, step, u, z);
  else if (rounds == 7)
    hipLaunchKernelGGL(rng_kernel<7>, grid, block, 0, s, key0, key1, stream_id, node0, count, step, u, z);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_swap_parity(int storage, const GatherArgs& g, void* tmp, hipStream_t s) {
  switch (storage) {
    case kF32: return swap_parity_words(g, static_cast<uint32_t*>(tmp), s);
    case kF16:
    case kBF16: return swap_parity_words(g, static_cast<uint16_t*>(tmp), s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const uint64_t n = bytes / sizeof(u32x4);
  if (n == 0) return hipSuccess;
  const uint64_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(copy_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s,
                     static_cast<u32x4*>(dst), static_cast<const u32x4*>(src), n);
  return hipGetLastError();
}

hipError_t launch_set_u32(uint32_t* dst, uint32_t value, hipStream_t s) {
  hipLaunchKernelGGL(set_u32_kernel, dim3(1), dim3(64), 0, s, dst, value);
  return hipGetLastError();
}

hipError_t launch_fill_zero(double* dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, dst,
                     static_cast<uint64_t>(n));
  return hipGetLastError();
}

}  // namespace rflbm
