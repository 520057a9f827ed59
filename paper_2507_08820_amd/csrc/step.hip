// step.hip -- the fused stream + collide step of the regularized fluctuating
// lattice Boltzmann method on D3Q27 (arXiv:2507.08820, Eq. r-flbe2), and the
// deterministic reduction of its ensemble statistics (Sec. III).
//
// One thread updates one node (the body is in node_body.inc):
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
//
// The same body runs in four kernels: step_kernel (tiles of 256 nodes of one z
// plane; every step shape, statistics included), step_wave_kernel (even steps
// in one-wave x-segments), step_row_kernel (odd steps in whole x-rows, where
// values move between lanes so that every access covers whole cache lines)
// and batch_kernel (many boxes, persistent grid over tiles of consecutive
// nodes).  The three one-box kernels take GEQ (every omega_g = 1) as a template
// parameter, and so does the batch kernel when every replica has it (else it
// reads the setting per replica).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "d3q27.hpp"
#include "fastdiv.hpp"
#include "kernels.hpp"
#include "philox.hpp"
#include "storage.hpp"

namespace rflbm {

namespace {

constexpr int kBlock = 256;

// Cache policy of the population accesses, per step parity.  The even step
// reads and writes each node's own slots: nothing is reused, so its loads are
// marked non-temporal.  The odd step reads and writes slots shifted by +-1 in
// x; neighbouring waves share the boundary cache lines, so its accesses keep
// the default policy and meet in L2.
#ifndef RFLBM_EVEN_LOAD_NT
#define RFLBM_EVEN_LOAD_NT 1
#endif
#ifndef RFLBM_EVEN_STORE_NT
#define RFLBM_EVEN_STORE_NT 1
#endif
#ifndef RFLBM_ODD_LOAD_NT
#define RFLBM_ODD_LOAD_NT 0
#endif
#ifndef RFLBM_ODD_STORE_NT
#define RFLBM_ODD_STORE_NT 0
#endif

// In the odd step the 9 populations with c_x = 0 are shifted only by whole
// rows, so their accesses do not share cache lines with neighbouring waves.
#ifndef RFLBM_ODD_ALIGNED_NT
#define RFLBM_ODD_ALIGNED_NT 0
#endif

// Cache policy of a population access of the tiled step; x_aligned (c_x = 0)
// is a constant once the population loop is unrolled.
template <bool ODD>
__device__ __forceinline__ constexpr bool load_nt(bool x_aligned) {
  return ODD ? (RFLBM_ODD_LOAD_NT || (x_aligned && RFLBM_ODD_ALIGNED_NT)) : RFLBM_EVEN_LOAD_NT;
}
template <bool ODD>
__device__ __forceinline__ constexpr bool store_nt(bool x_aligned) {
  return ODD ? (RFLBM_ODD_STORE_NT || (x_aligned && RFLBM_ODD_ALIGNED_NT == 1)) : RFLBM_EVEN_STORE_NT;
}

// Visiting order of the whole-row odd step: groups of 2 rows x 8 planes
// (measured at 512^3: about 1 % faster than plain row order).
#ifndef RFLBM_ROW_GROUP_Y
#define RFLBM_ROW_GROUP_Y 2
#define RFLBM_ROW_GROUP_Z 8
#endif

// x-row r = 0 .. ny nz - 1 of a visiting order -> (y, z).  With the row blocks
// in bricks, the bricks in memory order and y fastest inside each (a
// sequential walk of the populations; the odd step's 9 source and 9
// destination row blocks of a row lie in the brick of the row or its
// neighbours); otherwise rows in plane order.
__device__ __forceinline__ void brick_row(uint32_t r, const StepArgs& a, uint32_t& y, uint32_t& z) {
  const uint32_t inner = r & ((1u << (a.by_log + a.bz_log)) - 1u);
  const uint32_t brick = r >> (a.by_log + a.bz_log);
  const uint32_t zb = div_by(brick, a.ny >> a.by_log, a.div_nyb);
  const uint32_t yb = brick - zb * (a.ny >> a.by_log);
  y = (yb << a.by_log) + (inner & ((1u << a.by_log) - 1u));
  z = (zb << a.bz_log) + (inner >> a.by_log);
}

// Whole-row odd step: whole aligned cache lines that no other wave touches,
// like those of the even step.
#ifndef RFLBM_ROW_LOAD_NT
#define RFLBM_ROW_LOAD_NT 1
#endif
#ifndef RFLBM_ROW_STORE_NT
#define RFLBM_ROW_STORE_NT 1
#endif

// Population accesses are raw buffer instructions: a scalar resource (base
// address, no range limit below 4 GiB), a 32-bit per-lane offset and a scalar
// offset, so that no lane forms a 64-bit address.  Every offset sum stays
// below 4 GiB (the interface bounds one z plane, and a batch replica, to that).
typedef __amdgpu_buffer_rsrc_t BufRsrc;
constexpr int kBufferWord3 = 0x00020000;  // resource word 3 of raw buffers on gfx9-family targets
constexpr int kBufferNT = 2;              // cache-policy bit: non-temporal

template <class P>
__device__ __forceinline__ BufRsrc pop_rsrc(P base) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, 0, static_cast<int>(0xffffffffu), kBufferWord3);
}

template <class T>
__device__ __forceinline__ T buf_load(BufRsrc r, uint32_t voff, uint32_t soff, bool nt) {
  const int v = static_cast<int>(voff), s = static_cast<int>(soff);
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, nt ? __builtin_amdgcn_raw_buffer_load_b32(r, v, s, kBufferNT)
                                    : __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
  } else {
    const unsigned short b = nt ? __builtin_amdgcn_raw_buffer_load_b16(r, v, s, kBufferNT)
                                : __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0);
    return __builtin_bit_cast(T, b);
  }
}

template <class T>
__device__ __forceinline__ void buf_store(T q, BufRsrc r, uint32_t voff, uint32_t soff, bool nt) {
  const int v = static_cast<int>(voff), s = static_cast<int>(soff);
  if constexpr (sizeof(T) == 4) {
    const uint32_t b = __builtin_bit_cast(uint32_t, q);
    if (nt) __builtin_amdgcn_raw_buffer_store_b32(b, r, v, s, kBufferNT);
    else __builtin_amdgcn_raw_buffer_store_b32(b, r, v, s, 0);
  } else {
    const unsigned short b = __builtin_bit_cast(unsigned short, q);
    if (nt) __builtin_amdgcn_raw_buffer_store_b16(b, r, v, s, kBufferNT);
    else __builtin_amdgcn_raw_buffer_store_b16(b, r, v, s, 0);
  }
}

// Whole-wave lane shifts by one (DPP): lane l receives lane l - 1 (to_right)
// or lane l + 1 (to_left); the lane shifted in from outside the wave gets 0.
constexpr int kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138;
__device__ __forceinline__ uint32_t wave_shift_right(uint32_t v) {
  return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), kDppWaveShr1, 0xf, 0xf, false));
}
__device__ __forceinline__ uint32_t wave_shift_left(uint32_t v) {
  return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), kDppWaveShl1, 0xf, 0xf, false));
}

// Sum over the 64 lanes of a wave in a fixed order, by DPP lane moves: pairs and
// quads (quad permutations), half rows and rows of 16 (mirrors), then the four
// rows through the row broadcasts of lanes 15 and 31; the total ends in lane
// 63 and is returned to every lane (a scalar read).  Every move writes all
// rows, lanes without a source reading 0, so each add is one DPP instruction;
// only lane 63's chain (rows 2 + 3, then rows 0 + 1 from lane 31) is used.
constexpr int kDppQuadSwapPairs = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadSwapHalves = 0x4E;  // quad_perm [2, 3, 0, 1]
constexpr int kDppRowHalfMirror = 0x141, kDppRowMirror = 0x140;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

template <int CTRL>
__device__ __forceinline__ float dpp_add(float v) {
  const int moved = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true);
  return v + __int_as_float(moved);
}

__device__ __forceinline__ float wave_sum(float v) {
  v = dpp_add<kDppQuadSwapPairs>(v);
  v = dpp_add<kDppQuadSwapHalves>(v);
  v = dpp_add<kDppRowHalfMirror>(v);
  v = dpp_add<kDppRowMirror>(v);
  v = dpp_add<kDppRowBcast15>(v);
  v = dpp_add<kDppRowBcast31>(v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Whole-row blocks (blockDim.x = nx, so lane = x mod 64): replaces v[i], for
// every population with c_x = +-1, by the word that lane x - c_x holds.
// Inside a wave that is a shift by one lane; the one word per wave and
// population that crosses into the neighbouring wave (periodically, from the
// last wave into the first) goes through `edge` (18 x kMaxRowWaves words of
// LDS, used once per call site).  Ends with a block barrier.  Moving raw bit
// patterns keeps the arithmetic around the move identical to the tiled step's.
__device__ __forceinline__ void row_shift(uint32_t (&v)[kQ], uint32_t (*edge)[kMaxRowWaves], uint32_t x,
                                          uint32_t nx) {
  const uint32_t lane = x & 63u, wave = x >> 6, nwave = nx >> 6;
  // edge slot of population i with c_x = -1 (i = 3 k): 2 k; c_x = +1 (i = 3 k + 2): 2 k + 1
  if (lane == 63u) {
#pragma unroll
    for (int k = 0; k < 9; ++k) edge[2 * k + 1][wave] = v[3 * k + 2];
  }
  if (lane == 0u) {
#pragma unroll
    for (int k = 0; k < 9; ++k) edge[2 * k][wave] = v[3 * k];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    v[3 * k + 2] = wave_shift_right(v[3 * k + 2]);  // c_x = +1: from lane x - 1
    v[3 * k] = wave_shift_left(v[3 * k]);           // c_x = -1: from lane x + 1
  }
  __syncthreads();
  if (lane == 0u) {
    const uint32_t wprev = wave == 0 ? nwave - 1 : wave - 1;
#pragma unroll
    for (int k = 0; k < 9; ++k) v[3 * k + 2] = edge[2 * k + 1][wprev];
  }
  if (lane == 63u) {
    const uint32_t wnext = wave + 1 == nwave ? 0 : wave + 1;
#pragma unroll
    for (int k = 0; k < 9; ++k) v[3 * k] = edge[2 * k][wnext];
  }
}

// One box: a block covers bx x by nodes of one z plane (blockDim = (bx, by));
// blocks of one row (by = 1) take the rows in memory order, others plane by plane.
template <int S, bool ODD, int ROUNDS, bool STATS, bool GEQ>
__global__ void __launch_bounds__(kBlock) step_kernel(const StepArgs a) {
  uint32_t tile = blockIdx.x;
  if (a.xcd_remap) tile = (tile & 7u) * (gridDim.x >> 3) + (tile >> 3);
  const uint32_t rest = div_by(tile, a.tiles_x, a.div_tiles_x);
  const uint32_t tx = tile - rest * a.tiles_x;
  uint32_t y, z;
  if (blockDim.y == 1) {
    // tiles of one row: rows in memory order (brick by brick)
    brick_row(rest, a, y, z);
  } else {
    z = div_by(rest, a.tiles_y, a.div_tiles_y);
    y = (rest - z * a.tiles_y) * blockDim.y + threadIdx.y;
  }
  const uint32_t x = tx * blockDim.x + threadIdx.x;
  const uint32_t tid = threadIdx.x + blockDim.x * threadIdx.y;
  const bool active = tile < a.ntiles && x < a.nx && y < a.ny;

  __shared__ float stat_lds[STATS ? kNumStats : 1][kBlock];

  if (active) {
    const uint32_t step = a.step;
    constexpr bool STATS_WAVE = false;
    [[maybe_unused]] float (*stat_wave)[kMaxRowWaves] = nullptr;
    constexpr bool SMALL_BOX = false;
    constexpr bool BUFFER_ACCESS = true;
    constexpr bool BRICKS = true;
    constexpr bool ROW_SHIFT = false;
    constexpr bool GHOST_EQ = GEQ;
    [[maybe_unused]] uint32_t (*row_edge_in)[kMaxRowWaves] = nullptr;
    [[maybe_unused]] uint32_t (*row_edge_out)[kMaxRowWaves] = nullptr;
#include "node_body.inc"
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

// Even step without statistics in one-wave blocks: block b covers the 64
// nodes x = 64 (b mod (nx / 64)) + lane of x-row b / (nx / 64) of the memory
// order (brick_row; nx a multiple of 64).
template <int S, int ROUNDS, bool GEQ>
__global__ void __launch_bounds__(64) step_wave_kernel(const StepArgs a) {
  constexpr bool ODD = false, STATS = false, SMALL_BOX = false, ROW_SHIFT = false, BUFFER_ACCESS = true;
  constexpr bool BRICKS = true;
  constexpr bool GHOST_EQ = GEQ, STATS_WAVE = false;
  [[maybe_unused]] float (*stat_lds)[kBlock] = nullptr;
  [[maybe_unused]] float (*stat_wave)[kMaxRowWaves] = nullptr;
  [[maybe_unused]] const uint32_t tid = 0;
  [[maybe_unused]] uint32_t (*row_edge_in)[kMaxRowWaves] = nullptr;
  [[maybe_unused]] uint32_t (*row_edge_out)[kMaxRowWaves] = nullptr;
  uint32_t seg = blockIdx.x;
  if (a.xcd_remap) seg = (seg & 7u) * (gridDim.x >> 3) + (seg >> 3);
  const uint32_t per_row = a.nx >> 6;
  const uint32_t row = div_by(seg, per_row, a.div_segs);
  if (row >= a.ny * a.nz) return;  // the whole block: rounding of the grid to 8
  const uint32_t x = (seg - row * per_row) * 64 + threadIdx.x;
  uint32_t y, z;
  brick_row(row, a, y, z);
  const uint32_t step = a.step;
#include "node_body.inc"
}

// A step of one box in whole-row blocks: block b covers one x-row (blockDim.x
// = nx, a multiple of 64 up to 1024), rows in memory order (brick_row) or, in
// the plain layout, grouped on odd steps.  On odd
// steps the +-1 shifts in x stay inside the block and every load and store is
// a whole aligned cache line (see row_shift).  With STATS, each wave sums its
// nodes' statistics, and the block adds its waves' sums in FP64 (fixed order)
// into one partial per block, as step_kernel does; the even step takes this
// kernel only for statistics (one partial per row instead of one per wave).
template <int S, int ROUNDS, bool GEQ, bool STATS, bool ODD>
__global__ void __launch_bounds__(kMaxRowWaves * 64) step_row_kernel(const StepArgs a) {
  constexpr bool SMALL_BOX = false, ROW_SHIFT = ODD, BUFFER_ACCESS = true, BRICKS = true;
  constexpr bool GHOST_EQ = GEQ, STATS_WAVE = true;
  [[maybe_unused]] float (*stat_lds)[kBlock] = nullptr;
  [[maybe_unused]] const uint32_t tid = 0;
  __shared__ uint32_t row_edge_in[18][kMaxRowWaves];   // gather (stored words)
  __shared__ uint32_t row_edge_out[18][kMaxRowWaves];  // scatter (FP32 values)
  __shared__ float stat_wave[STATS ? kNumStats : 1][kMaxRowWaves];
  uint32_t row = blockIdx.x;
  if (a.xcd_remap) row = (row & 7u) * (gridDim.x >> 3) + (row >> 3);
  if (row >= a.ny * a.nz) {  // the whole block: rounding of the grid to 8
    if constexpr (STATS) {
      if (threadIdx.x < kNumStats) a.partials[static_cast<size_t>(threadIdx.x) * gridDim.x + blockIdx.x] = 0.0;
    }
    return;
  }
  const uint32_t x = threadIdx.x;
  uint32_t y, z;
  if (a.by_log + a.bz_log > 0) {
    brick_row(row, a, y, z);
  } else {
#if RFLBM_ROW_GROUP_Y * RFLBM_ROW_GROUP_Z > 1
    // plain layout, odd steps: rows visited in groups of GY x GZ (y, z) so
    // that the 9 row blocks a row reads from and writes to are in use at
    // about the same time
    constexpr uint32_t GY = ODD ? RFLBM_ROW_GROUP_Y : 1, GZ = ODD ? RFLBM_ROW_GROUP_Z : 1;
    const uint32_t per_zgroup = a.ny * GZ;
    const uint32_t zg = row / per_zgroup;
    const uint32_t r2 = row - zg * per_zgroup;
    const uint32_t gzh = min(GZ, a.nz - zg * GZ);
    const uint32_t yg = r2 / (GY * gzh);
    const uint32_t r3 = r2 - yg * GY * gzh;
    const uint32_t gyw = min(GY, a.ny - yg * GY);
    y = yg * GY + r3 % gyw;
    z = zg * GZ + r3 / gyw;
#else
    y = row % a.ny;
    z = row / a.ny;
#endif
  }
  const uint32_t step = a.step;
#include "node_body.inc"
  if constexpr (STATS) {
    __syncthreads();
    if (x < kNumStats) {
      double acc = 0.0;
      for (uint32_t w = 0; w < (a.nx >> 6); ++w) acc += static_cast<double>(stat_wave[x][w]);
      a.partials[static_cast<size_t>(x) * gridDim.x + blockIdx.x] = acc;
    }
  }
}

// Many boxes: tile t holds blockDim.x consecutive nodes (flattened index) of
// replica tile_rep[t]; a persistent grid walks the tiles.  The step count (the
// Philox counter) is the device counter plus b.step_offset, so that a captured
// graph of several steps (offsets 0, 1, ...) can be replayed from any t; the
// parity is a template parameter, and the host only replays graphs of an even
// number of steps from an even step count.  GEQ: every replica has every
// omega_g = 1; otherwise each replica's own setting is read at run time.
// STATS: each tile's statistics are reduced in the block (fixed order, FP64)
// into column t of b.partials, for batch_stats_reduce.
template <int S, bool ODD, int ROUNDS, bool GEQ, bool STATS>
__global__ void __launch_bounds__(kBlock) batch_kernel(const BatchArgs b) {
  constexpr bool STATS_WAVE = false;
  [[maybe_unused]] float (*stat_wave)[kMaxRowWaves] = nullptr;
  constexpr bool SMALL_BOX = true;  // every replica region is below 4 GiB
  constexpr bool BRICKS = false;    // replicas keep the plain layout
  // buffer instructions measured faster for 16-bit storage, global ones for
  // FP32 (64 replicas of 32^3..96^3: 38.9 vs 36.6 and 24.6 vs 25.9 GLUPS)
  constexpr bool BUFFER_ACCESS = S != kF32;
  constexpr bool ROW_SHIFT = false;
  [[maybe_unused]] uint32_t (*row_edge_in)[kMaxRowWaves] = nullptr;
  [[maybe_unused]] uint32_t (*row_edge_out)[kMaxRowWaves] = nullptr;
  __shared__ float stat_lds[STATS ? kNumStats : 1][kBlock];
  __shared__ double stat_part[STATS ? kNumStats : 1][kBlock / 32];
  const uint32_t tid = threadIdx.x;
  // the tables are read-only for the whole launch: constant address space,
  // so the per-tile lookups are scalar loads
  typedef __attribute__((address_space(4))) const ReplicaArgs CReps;
  typedef __attribute__((address_space(4))) const uint32_t CU32;
  CReps* const reps = (CReps*)(b.reps);
  CU32* const tile_rep = (CU32*)(b.tile_rep);
  const uint32_t step = *(CU32*)(b.step) + b.step_offset;
  for (uint32_t tile = blockIdx.x; tile < b.ntiles; tile += gridDim.x) {
    CReps& r = reps[tile_rep[tile]];
    __attribute__((address_space(4))) const StepArgs& a = r.a;
    const uint32_t n = (tile - r.tile0) * blockDim.x + threadIdx.x;
    if (n < r.nodes) {
      const uint32_t z = fast_div(n, FastDiv{r.div_xy.m, r.div_xy.s});
      const uint32_t rem = n - z * (a.nx * a.ny);
      const uint32_t y = fast_div(rem, FastDiv{r.div_x.m, r.div_x.s});
      const uint32_t x = rem - y * a.nx;
      const bool GHOST_EQ = GEQ || a.ghost_eq != 0u;
#include "node_body.inc"
    } else if constexpr (STATS) {
#pragma unroll
      for (int c = 0; c < kNumStats; ++c) stat_lds[c][tid] = 0.0f;
    }
    if constexpr (STATS) {
      // parts of 32 nodes per column, then the parts in order, in FP64
      const uint32_t parts = blockDim.x / 32;
      __syncthreads();
      if (tid < kNumStats * parts) {
        const uint32_t c = tid / parts, p = tid - c * parts;
        double acc = 0.0;
#pragma unroll 8
        for (int e = 0; e < 32; ++e) acc += static_cast<double>(stat_lds[c][p * 32 + e]);
        stat_part[c][p] = acc;
      }
      __syncthreads();
      if (tid < kNumStats) {
        double acc = 0.0;
        for (uint32_t p = 0; p < parts; ++p) acc += stat_part[tid][p];
        b.partials[static_cast<size_t>(tid) * b.partial_pitch + tile] = acc;
      }
      __syncthreads();  // stat_lds is refilled by the block's next tile
    }
  }
}

// Statistics of a batch step: block r adds the tile partials of replica r in
// tile order (8 strided parts per column, then the parts in order, FP64) and
// accumulates them into the replica's accumulators like accumulate_stats.
__global__ void __launch_bounds__(256) batch_stats_reduce(const BatchArgs b, uint32_t tile_nodes) {
  const ReplicaArgs& r = b.reps[blockIdx.x];
  const uint32_t ntiles = (r.nodes + tile_nodes - 1) / tile_nodes;
  __shared__ double part[kNumStats][8];
  const uint32_t tid = threadIdx.x;
  if (tid < kNumStats * 8) {
    const uint32_t c = tid >> 3, p = tid & 7;
    const double* col = b.partials + static_cast<size_t>(c) * b.partial_pitch + r.tile0;
    double acc = 0.0;
    for (uint32_t k = p; k < ntiles; k += 8) acc += col[k];
    part[c][p] = acc;
  }
  __syncthreads();
  if (tid < kNumStats) {
    double sum = 0.0;
#pragma unroll
    for (int p = 0; p < 8; ++p) sum += part[tid][p];
    r.acc[tid] += sum;
    if (tid == 0) r.acc[kNumStats] += 1.0;
    if (tid == 0) r.acc[kNumStats + 1] = sum;                          // mass deviation
    if (tid >= 2 && tid <= 4) r.acc[kNumStats + tid] = sum;            // momentum
  }
}

__global__ void advance_step(uint32_t* step, uint32_t delta) {
  if (threadIdx.x == 0) *step += delta;
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
  if (a.ghost_eq)
    hipLaunchKernelGGL((step_kernel<S, ODD, R, ST, true>), dim3(l.grid), dim3(l.bx, l.by), 0, s, a);
  else
    hipLaunchKernelGGL((step_kernel<S, ODD, R, ST, false>), dim3(l.grid), dim3(l.bx, l.by), 0, s, a);
  return hipGetLastError();
}

template <int S, int R, bool ST, bool ODD>
void launch_row_g(const StepArgs& a, dim3 g, dim3 blk, hipStream_t s) {
  if (a.ghost_eq) hipLaunchKernelGGL((step_row_kernel<S, R, true, ST, ODD>), g, blk, 0, s, a);
  else hipLaunchKernelGGL((step_row_kernel<S, R, false, ST, ODD>), g, blk, 0, s, a);
}

template <int S, int R>
void launch_wave_g(const StepArgs& a, dim3 g, hipStream_t s) {
  if (a.ghost_eq) hipLaunchKernelGGL((step_wave_kernel<S, R, true>), g, dim3(64), 0, s, a);
  else hipLaunchKernelGGL((step_wave_kernel<S, R, false>), g, dim3(64), 0, s, a);
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

template <int S, bool ST, bool ODD>
hipError_t launch_row_s(int rounds, const StepArgs& a, uint32_t grid, hipStream_t s) {
  const dim3 g(grid), blk(a.nx);
  switch (rounds) {
    case 0: launch_row_g<S, 0, ST, ODD>(a, g, blk, s); break;
    case 7: launch_row_g<S, 7, ST, ODD>(a, g, blk, s); break;
    case 10: launch_row_g<S, 10, ST, ODD>(a, g, blk, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The even whole-row kernel runs only with statistics.
template <int S>
hipError_t launch_row_st(bool odd, bool stats, int rounds, const StepArgs& a, uint32_t grid, hipStream_t s) {
  if (!odd) return stats ? launch_row_s<S, true, false>(rounds, a, grid, s) : hipErrorInvalidConfiguration;
  return stats ? launch_row_s<S, true, true>(rounds, a, grid, s) : launch_row_s<S, false, true>(rounds, a, grid, s);
}

template <int S>
hipError_t launch_wave_s(int rounds, const StepArgs& a, uint32_t grid, hipStream_t s) {
  switch (rounds) {
    case 0: launch_wave_g<S, 0>(a, dim3(grid), s); break;
    case 7: launch_wave_g<S, 7>(a, dim3(grid), s); break;
    case 10: launch_wave_g<S, 10>(a, dim3(grid), s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step_wave(int storage, int rounds, const StepArgs& a, hipStream_t stream) {
  if (a.nx % 64 != 0 || a.nx == 0) return hipErrorInvalidConfiguration;
  const uint64_t segs = static_cast<uint64_t>(a.nx / 64) * a.ny * a.nz;
  if (segs >= (1ull << 31)) return hipErrorInvalidConfiguration;
  const uint32_t grid = static_cast<uint32_t>((segs + 7) / 8 * 8);
  switch (storage) {
    case kF32: return launch_wave_s<kF32>(rounds, a, grid, stream);
    case kF16: return launch_wave_s<kF16>(rounds, a, grid, stream);
    case kBF16: return launch_wave_s<kBF16>(rounds, a, grid, stream);
    default: return hipErrorInvalidValue;
  }
}

bool row_kernel_fits(uint32_t nx) { return nx % 64 == 0 && nx >= 64 && nx <= kMaxRowWaves * 64; }

uint32_t row_grid(uint32_t ny, uint32_t nz) {
  const uint64_t rows = static_cast<uint64_t>(ny) * nz;
  return static_cast<uint32_t>((rows + 7) / 8 * 8);
}

hipError_t launch_step_row(int storage, bool odd, int rounds, bool stats, const StepArgs& a, hipStream_t stream) {
  if (!row_kernel_fits(a.nx)) return hipErrorInvalidConfiguration;
  const uint64_t rows = static_cast<uint64_t>(a.ny) * a.nz;
  if (rows >= (1ull << 31)) return hipErrorInvalidConfiguration;
  const uint32_t grid = row_grid(a.ny, a.nz);
  switch (storage) {
    case kF32: return launch_row_st<kF32>(odd, stats, rounds, a, grid, stream);
    case kF16: return launch_row_st<kF16>(odd, stats, rounds, a, grid, stream);
    case kBF16: return launch_row_st<kBF16>(odd, stats, rounds, a, grid, stream);
    default: return hipErrorInvalidValue;
  }
}

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

hipError_t launch_batch_step(int storage, bool odd, int rounds, bool all_ghost_eq, bool stats,
                             const BatchArgs& b, uint32_t grid, uint32_t tile, hipStream_t stream) {
  if (tile != 128 && tile != 256) return hipErrorInvalidConfiguration;
  if (stats && !b.partials) return hipErrorInvalidValue;
  const dim3 g(grid), blk(tile);
#define RFLBM_BATCH_ST(S, O, R, G)                                                             \
  if (stats)                                                                                   \
    hipLaunchKernelGGL((batch_kernel<S, O, R, G, true>), g, blk, 0, stream, b);                \
  else                                                                                         \
    hipLaunchKernelGGL((batch_kernel<S, O, R, G, false>), g, blk, 0, stream, b);
#define RFLBM_BATCH_G(S, O, R)                                                                 \
  if (all_ghost_eq) {                                                                          \
    RFLBM_BATCH_ST(S, O, R, true)                                                              \
  } else {                                                                                     \
    RFLBM_BATCH_ST(S, O, R, false)                                                             \
  }
#define RFLBM_BATCH_R(S, O)                                                                    \
  switch (rounds) {                                                                            \
    case 0: RFLBM_BATCH_G(S, O, 0) break;                                                      \
    case 7: RFLBM_BATCH_G(S, O, 7) break;                                                      \
    case 10: RFLBM_BATCH_G(S, O, 10) break;                                                    \
    default: return hipErrorInvalidValue;                                                      \
  }
#define RFLBM_BATCH(S)            \
  if (odd) {                      \
    RFLBM_BATCH_R(S, true)        \
  } else {                        \
    RFLBM_BATCH_R(S, false)       \
  }
  switch (storage) {
    case kF32: RFLBM_BATCH(kF32) break;
    case kF16: RFLBM_BATCH(kF16) break;
    case kBF16: RFLBM_BATCH(kBF16) break;
    default: return hipErrorInvalidValue;
  }
#undef RFLBM_BATCH
#undef RFLBM_BATCH_R
#undef RFLBM_BATCH_G
#undef RFLBM_BATCH_ST
  return hipGetLastError();
}

hipError_t launch_batch_stats_reduce(const BatchArgs& b, uint32_t nrep, uint32_t tile, hipStream_t stream) {
  if (nrep == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_stats_reduce, dim3(nrep), dim3(256), 0, stream, b, tile);
  return hipGetLastError();
}

hipError_t launch_advance_step(uint32_t* step, uint32_t delta, hipStream_t stream) {
  hipLaunchKernelGGL(advance_step, dim3(1), dim3(64), 0, stream, step, delta);
  return hipGetLastError();
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
