// step.hip -- the fused stream + collide step of the regularized fluctuating
// lattice Boltzmann method on D3Q27 (arXiv:2507.08820, Eq. r-flbe2), and the
// deterministic reduction of its ensemble statistics (Sec. III).
//
// One thread updates one node:
//   1. gather the 27 populations arriving at x (AA pattern, see kernels.hpp);
//   2. project them on the Table II Hermite modes (Eq. moments) with three
//      3-point sweeps (d3q27.hpp);
//   3. [statistics steps] stage rho, j, u^2, Pi and their squares in LDS;
//   4. rebuild the equilibrium modes m_eq = rho u_x^px u_y^py u_z^pz, the
//      recursive coefficients a0^(n) = a0^(n-1) u of Eq. rec-eq;
//   5. relax the non-equilibrium part a = m - m_eq: the deviatoric
//      second-order modes with omega_s, the trace of {xx, yy, zz} with omega_b,
//      the ghosts k = 10..26 with omega_g (paper: omega_b = omega_s = omega_h,
//      omega_g = 1, where the ghost non-equilibrium vanishes);
//   6. add phi_k r_k to every mode k = 4..26 (Eq. fluct_phi, local density),
//      r_k from Philox4x32 + Box-Muller (philox.hpp);
//   7. transform back (Eq. backtrasf) and scatter the 27 post-collision
//      values to their AA destination slots.
// Everything between the 27 loads and the 27 stores stays in registers.
#include <hip/hip_runtime.h>

#include "d3q27.hpp"
#include "kernels.hpp"
#include "philox.hpp"
#include "storage.hpp"

namespace rflbm {

namespace {

constexpr int kBlock = 256;

template <int S, bool ODD, int ROUNDS, bool STATS>
__global__ void __launch_bounds__(kBlock) step_kernel(const StepArgs a) {
  using C = Codec<S>;
  using T = typename C::T;

  uint32_t tile = blockIdx.x;
  if (a.xcd_remap) tile = (tile & 7u) * (gridDim.x >> 3) + (tile >> 3);
  const uint32_t tx = tile % a.tiles_x;
  const uint32_t rest = tile / a.tiles_x;
  const uint32_t ty = rest % a.tiles_y;
  const uint32_t z = rest / a.tiles_y;
  const uint32_t x = tx * blockDim.x + threadIdx.x;
  const uint32_t y = ty * blockDim.y + threadIdx.y;
  const uint32_t tid = threadIdx.x + blockDim.x * threadIdx.y;
  const bool active = tile < a.ntiles && x < a.nx && y < a.ny;

  __shared__ float stat_lds[STATS ? kNumStats : 1][STATS ? kBlock : 1];

  if (active) {
    const uint32_t nx = a.nx, ny = a.ny, nz = a.nz, sxy = nx * ny;
    // byte offsets of the three x, y, z coordinates x - 1, x, x + 1 (periodic)
    uint32_t X[3], Y[3], Z[3];
    X[0] = wrap_add(x, -1, nx) * sizeof(T);
    X[1] = x * sizeof(T);
    X[2] = wrap_add(x, 1, nx) * sizeof(T);
    Y[0] = wrap_add(y, -1, ny) * nx * sizeof(T);
    Y[1] = y * nx * sizeof(T);
    Y[2] = wrap_add(y, 1, ny) * nx * sizeof(T);
    Z[0] = wrap_add(z, -1, nz) * sxy * sizeof(T);
    Z[1] = z * sxy * sizeof(T);
    Z[2] = wrap_add(z, 1, nz) * sxy * sizeof(T);
    const uint64_t plane_bytes = a.pitch * sizeof(T);
    char* const base = static_cast<char*>(a.pop);

    // 1. gather
    float v[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int ix = i % 3, iy = (i / 3) % 3, iz = i / 9;
      const int plane = ODD ? kQ - 1 - i : i;
      const uint32_t off = ODD ? X[2 - ix] + Y[2 - iy] + Z[2 - iz] : X[1] + Y[1] + Z[1];
      const T q = *reinterpret_cast<const T*>(base + plane * plane_bytes + off);
      v[i] = C::decode(q, a.sigma[speed_class(i)]);
    }

    // 2. Hermite projection (deviation form: slot 0 holds rho - rho0)
    forward27(v);
    const float rho = a.rho0 + v[0];
    const float inv_rho = __builtin_amdgcn_rcpf(rho);
    const float ux = v[1] * inv_rho, uy = v[3] * inv_rho, uz = v[9] * inv_rho;
    if (!(rho > 0.0f) || !(fabsf(ux) + fabsf(uy) + fabsf(uz) < 1.0e30f)) *a.flag = 1;

    // 3. statistics of the pre-collision state
    if constexpr (STATS) {
      const float s[kNumStats] = {
          v[0], v[0] * v[0],
          v[1], v[3], v[9], v[1] * v[1], v[3] * v[3], v[9] * v[9],
          ux * ux, uy * uy, uz * uz,
          v[2], v[6], v[18], v[4], v[10], v[12],
          v[2] * v[2], v[6] * v[6], v[18] * v[18], v[4] * v[4], v[10] * v[10], v[12] * v[12]};
#pragma unroll
      for (int c = 0; c < kNumStats; ++c) stat_lds[c][tid] = s[c];
    }

    // 4. equilibrium modes m_eq(px, py, pz) = exy[px + 3 py] * ez[pz]
    float exy[9];
    {
      const float ex[3] = {1.0f, ux, ux * ux};
      const float ey[3] = {1.0f, uy, uy * uy};
#pragma unroll
      for (int py = 0; py < 3; ++py)
#pragma unroll
        for (int px = 0; px < 3; ++px) exy[px + 3 * py] = ex[px] * ey[py];
    }
    const float ez[3] = {rho, rho * uz, rho * uz * uz};
    auto meq = [&](int slot) -> float { return slot < 9 ? exy[slot] * rho : exy[slot % 9] * ez[slot / 9]; };

    // 5. relaxation of the non-equilibrium modes
    {
      const int sxx = mode_slot(4), syy = mode_slot(5), szz = mode_slot(6);
      const float exx = meq(sxx), eyy = meq(syy), ezz = meq(szz);
      const float axx = v[sxx] - exx, ayy = v[syy] - eyy, azz = v[szz] - ezz;
      const float tr = (axx + ayy + azz) * (1.0f / 3.0f) * a.lam_b_minus_s;
      v[sxx] = exx + fmaf(a.lam_s, axx, tr);
      v[syy] = eyy + fmaf(a.lam_s, ayy, tr);
      v[szz] = ezz + fmaf(a.lam_s, azz, tr);
    }
#pragma unroll
    for (int k = 7; k <= 9; ++k) {
      const int s = mode_slot(k);
      const float e = meq(s);
      v[s] = fmaf(a.lam_s, v[s] - e, e);
    }
#pragma unroll
    for (int k = 10; k < kQ; ++k) {
      const int s = mode_slot(k);
      const float e = meq(s);
      v[s] = fmaf(a.lam_g[k - 10], v[s] - e, e);
    }

    // 6. noise phi_k r_k, phi_k = sqrt(rho) * amp_k
    if constexpr (ROUNDS > 0) {
      const float srho = __builtin_amdgcn_sqrtf(rho);
      const uint32_t node = (X[1] + Y[1] + Z[1]) / sizeof(T);
#pragma unroll
      for (uint32_t j = 0; j < 6; ++j) {
        const Word4 w = philox<ROUNDS>(Word4{node, a.step, j, a.stream_id}, a.key0, a.key1);
        float r[4];
        box_muller(w.w0, w.w1, r[0], r[1]);
        box_muller(w.w2, w.w3, r[2], r[3]);
        if (j == 0) {
          const float rbar = (r[0] + r[1] + r[2]) * (1.0f / 3.0f);
          const float tr = srho * a.amp_b_minus_s * rbar;
          const float sd = srho * a.amp_s;
          v[mode_slot(4)] += fmaf(sd, r[0], tr);
          v[mode_slot(5)] += fmaf(sd, r[1], tr);
          v[mode_slot(6)] += fmaf(sd, r[2], tr);
          v[mode_slot(7)] = fmaf(srho * a.amp_off, r[3], v[mode_slot(7)]);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int k = 4 + 4 * static_cast<int>(j) + q;
            if (k < kQ) {
              const float amp = k <= 9 ? a.amp_off : a.amp_g[k - 10];
              v[mode_slot(k)] = fmaf(srho * amp, r[q], v[mode_slot(k)]);
            }
          }
        }
      }
    }

    // 7. back to populations (slot 0 still holds rho - rho0) and scatter
    inverse27(v);
    // The even step stores at the offset it loaded from.  Hiding that equality
    // from the compiler keeps it from holding 27 64-bit load addresses live
    // across the collision; every access then uses a scalar plane base plus a
    // 32-bit vector offset.
    uint32_t own = X[1] + Y[1] + Z[1];
    if constexpr (!ODD) asm volatile("" : "+v"(own));
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int ix = i % 3, iy = (i / 3) % 3, iz = i / 9;
      const int plane = ODD ? i : kQ - 1 - i;
      const uint32_t off = ODD ? X[ix] + Y[iy] + Z[iz] : own;
      T* dst = reinterpret_cast<T*>(base + plane * plane_bytes + off);
      __builtin_nontemporal_store(C::encode(v[i], a.inv_sigma[speed_class(i)]), dst);
    }
  } else if constexpr (STATS) {
#pragma unroll
    for (int c = 0; c < kNumStats; ++c) stat_lds[c][tid] = 0.0f;
  }

  if constexpr (STATS) {
    // fixed-order block reduction in FP64: 8 partial sums of 32 nodes per column
    __shared__ double part[kNumStats][8];
    __syncthreads();
    if (tid < kNumStats * 8) {
      const int c = tid >> 3, p = tid & 7;
      double acc = 0.0;
#pragma unroll 8
      for (int e = 0; e < 32; ++e) acc += static_cast<double>(stat_lds[c][p * 32 + e]);
      part[c][p] = acc;
    }
    __syncthreads();
    if (tid < kNumStats) {
      double acc = 0.0;
#pragma unroll
      for (int p = 0; p < 8; ++p) acc += part[tid][p];
      a.partials[static_cast<size_t>(tid) * gridDim.x + blockIdx.x] = acc;
    }
  }
}

// Sums 2048 consecutive entries of one column per block (fixed order).
constexpr uint32_t kReduceChunk = 2048;

__global__ void __launch_bounds__(256) reduce_columns(const double* in, uint32_t n_in, double* out,
                                                      uint32_t n_out) {
  const double* col = in + static_cast<size_t>(blockIdx.y) * n_in;
  const uint32_t base = blockIdx.x * kReduceChunk;
  double acc = 0.0;
#pragma unroll
  for (uint32_t k = 0; k < kReduceChunk / 256; ++k) {
    const uint32_t i = base + k * 256 + threadIdx.x;
    if (i < n_in) acc += col[i];
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (uint32_t s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[static_cast<size_t>(blockIdx.y) * n_out + blockIdx.x] = sh[0];
}

// acc[0..22] += sums; acc[23] += 1 (samples); acc[24] = mass; acc[25..27] = momentum.
__global__ void accumulate_stats(const double* sums, double* acc) {
  const int c = threadIdx.x;
  if (c < kNumStats) acc[c] += sums[c];
  if (c == 0) {
    acc[kNumStats] += 1.0;
    acc[kNumStats + 1] = sums[0];
    acc[kNumStats + 2] = sums[2];
    acc[kNumStats + 3] = sums[3];
    acc[kNumStats + 4] = sums[4];
  }
}

template <int S, bool ODD, int R, bool ST>
hipError_t launch_t(const StepArgs& a, const Launch& l, hipStream_t s) {
  hipLaunchKernelGGL((step_kernel<S, ODD, R, ST>), dim3(l.grid), dim3(l.bx, l.by), 0, s, a);
  return hipGetLastError();
}

template <int S, bool ODD, bool ST>
hipError_t launch_r(int rounds, const StepArgs& a, const Launch& l, hipStream_t s) {
  switch (rounds) {
    case 0: return launch_t<S, ODD, 0, ST>(a, l, s);
    case 7: return launch_t<S, ODD, 7, ST>(a, l, s);
    case 10: return launch_t<S, ODD, 10, ST>(a, l, s);
    default: return hipErrorInvalidValue;
  }
}

template <int S>
hipError_t launch_s(bool odd, int rounds, bool stats, const StepArgs& a, const Launch& l,
                    hipStream_t s) {
  if (odd) return stats ? launch_r<S, true, true>(rounds, a, l, s) : launch_r<S, true, false>(rounds, a, l, s);
  return stats ? launch_r<S, false, true>(rounds, a, l, s) : launch_r<S, false, false>(rounds, a, l, s);
}

}  // namespace

Launch make_launch(uint32_t nx, uint32_t ny, uint32_t nz, uint32_t bx, uint32_t by) {
  Launch l;
  l.bx = bx;
  l.by = by;
  const uint64_t tiles = static_cast<uint64_t>((nx + bx - 1) / bx) * ((ny + by - 1) / by) * nz;
  l.grid = static_cast<uint32_t>((tiles + 7) / 8 * 8);
  return l;
}

hipError_t launch_step(int storage, bool odd, int rounds, bool stats, const StepArgs& a,
                       const Launch& l, hipStream_t stream) {
  if (l.bx * l.by != kBlock || l.bx % 64 != 0 || l.grid % 8 != 0) return hipErrorInvalidConfiguration;
  switch (storage) {
    case kF32: return launch_s<kF32>(odd, rounds, stats, a, l, stream);
    case kF16: return launch_s<kF16>(odd, rounds, stats, a, l, stream);
    case kBF16: return launch_s<kBF16>(odd, rounds, stats, a, l, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_stats_reduce(const double* partials, uint32_t grid, double* scratch, double* acc,
                               hipStream_t stream) {
  const double* in = partials;
  uint32_t n = grid;
  double* bufs[2] = {scratch, scratch + static_cast<size_t>(kNumStats) *
                                            ((grid + kReduceChunk - 1) / kReduceChunk)};
  int which = 0;
  while (n > 1) {
    const uint32_t n_out = (n + kReduceChunk - 1) / kReduceChunk;
    hipLaunchKernelGGL(reduce_columns, dim3(n_out, kNumStats), dim3(256), 0, stream, in, n,
                       bufs[which], n_out);
    in = bufs[which];
    which ^= 1;
    n = n_out;
  }
  hipLaunchKernelGGL(accumulate_stats, dim3(1), dim3(64), 0, stream, in, acc);
  return hipGetLastError();
}

}  // namespace rflbm
