// kernels.hpp -- internal interface between the C-ABI layer (api.cpp) and the HIP
// kernels of the fluctuating lattice Boltzmann step (arXiv:2507.08820, Sec. II).
//
// Population storage ("AA" in-place streaming, one lattice copy), blocked by
// x-rows: the 27 population rows of the x-row (y, z) are contiguous (an x-row
// block), element (i, x) of it at offset i Q + x, population-row pitch Q >= nx.
// The row blocks themselves are stored in bricks of By x Bz rows (y fastest
// inside a brick), the bricks y-major within a brick row of Bz planes:
//   block(y, z) = Y(y) + Z(z),
//   Y(y) = (y / By) Yb + (y mod By) R,   Z(z) = (z / Bz) P + (z mod Bz) Zi,
// with R >= 27 Q, Zi = By R, Yb = By Bz R and P >= (ny / By) Yb (By, Bz
// powers of two dividing ny and nz; By = Bz = 1 is the plain layout, rows
// y-major within planes, P the plane pitch).  A[i][n] below names slot (i, x)
// of the row block of node n = x + nx (y + ny z).  Each slot holds the
// deviation f - w_i rho0 (divided by sigma_class(i) for 16-bit storage).
//   After an even number t of steps: f_i(x, t) = A[i][x].
//   After an odd number t of steps:  f_i(x, t) = A[26 - i][x - c_i].
// An even step reads A[i][x] and writes f*_i(x) to A[26 - i][x]; an odd step
// reads A[26 - i][x - c_i] and writes f*_i(x) to A[i][x + c_i].  In both cases
// every slot is read and then written by the same thread, so the update is
// race free in place, and the stored state after the step is the streamed
// f(t + 1) of Eq. eq:streaming.
#pragma once
#include <cstdint>
#include <hip/hip_runtime.h>

#include "fastdiv.hpp"

namespace rflbm {

enum Storage : int { kF32 = 0, kF16 = 1, kBF16 = 2 };

constexpr uint32_t kMaxRowWaves = 16;  // whole-row odd step: nx <= 1024
constexpr int kNumStats = 23;  // per-node statistics accumulated by the step kernel
// column layout: 0 drho, 1 drho^2, 2-4 j, 5-7 j^2, 8-10 u^2, 11-16 Pi, 17-22 Pi^2
constexpr int kAccDoubles = 32;  // device accumulator block: 23 sums, samples, mass, momentum

struct StepArgs {
  void* pop;             // populations, x-row blocked
  uint32_t nx, ny, nz;   // box
  uint32_t pop_pitch;    // bytes from population row i to row i + 1 of one x-row block (Q)
  uint32_t row_pitch;    // bytes from one x-row block to the next in y inside a brick (R)
  uint32_t ybrick_pitch; // bytes from one brick to the next in y (Yb; R when By = 1)
  uint32_t zin_pitch;    // bytes from one x-row block to the next in z inside a brick (Zi)
  uint32_t by_log, bz_log;  // log2 of the brick shape By x Bz (0, 0: plain layout)
  uint64_t plane_pitch;  // bytes from one brick row (Bz z planes) to the next (P)
  uint32_t tiles_x;      // tiles along x (tile = blockDim.x x blockDim.y nodes of one z plane)
  uint32_t tiles_y;      // tiles along y
  uint32_t ntiles;       // tiles_x * tiles_y * nz
  uint32_t xcd_remap;    // 1: give each XCD a contiguous range of tiles
  FastDiv div_tiles_x;   // division by tiles_x (when tiles_x >= 2)
  FastDiv div_tiles_y;   // division by tiles_y (when tiles_y >= 2)
  FastDiv div_ny;        // division by ny
  FastDiv div_nyb;       // division by ny / By (bricks along y)
  FastDiv div_segs;      // division by nx / 64 (when nx / 64 >= 2)
  uint32_t step;         // t mod 2^32 (Philox counter word 1)
  uint32_t key0, key1;   // Philox key
  uint32_t stream_id;    // Philox counter word 3
  float rho0;
  float lam_s;           // 1 - omega_s (deviatoric second-order modes)
  float lam_b_minus_s;   // (1 - omega_b) - (1 - omega_s) (trace of the xx, yy, zz block)
  // noise amplitudes, each multiplied by inv_scale of its mode's register slot
  // (d3q27.hpp), the scale the step kernels carry the modes in
  float amp_s;           // sqrt(kT b_4 / cs2) s(omega_s), s(w) = sqrt(w (2 - w)); modes 4..6
  float amp_b_minus_s;   // sqrt(kT b_4 / cs2) (s(omega_b) - s(omega_s))
  float amp_off;         // sqrt(kT b_7 / cs2) s(omega_s), modes 7..9
  uint32_t ghost_eq;     // 1 when every omega_g,k = 1 (all lam_g = 0)
  uint32_t ghost_rec;    // 1: ghosts relax the coefficients Eq. recursive_eq rebuilds
                         // from the second-order ones and u (else the projected ones)
  float lam_g[17];       // 1 - omega_g,k, k = 10..26
  float amp_g[17];       // sqrt(kT b_k / cs2) s(omega_g,k)
  float sigma[4];        // storage unit per speed class (1 for FP32)
  float inv_sigma[4];
  int* flag;             // set to 1 on rho <= 0 or non-finite rho, j
  double* partials;      // statistics partials, column-major [kNumStats][gridDim.x]
};

// Byte offsets of the row block of (y, z): the y part Y(y) and the z part Z(z)
// of the brick layout above.
// (A: StepArgs in any address space.)
template <class A>
__host__ __device__ __forceinline__ uint32_t row_off_y(uint32_t y, const A& a) {
  return (y >> a.by_log) * a.ybrick_pitch + (y & ((1u << a.by_log) - 1u)) * a.row_pitch;
}
template <class A>
__host__ __device__ __forceinline__ uint64_t row_off_z(uint32_t z, const A& a) {
  return static_cast<uint64_t>(z >> a.bz_log) * a.plane_pitch +
         static_cast<uint64_t>((z & ((1u << a.bz_log) - 1u)) * a.zin_pitch);
}

// One replica of a batch: its lattice arguments plus what the batched kernel
// needs to turn a tile-local flattened node index into (x, y, z).
struct ReplicaArgs {
  StepArgs a;        // layout and physics of the replica (tiling fields unused)
  uint32_t tile0;    // first tile of the replica in the batch's tile list
  uint32_t nodes;    // nx * ny * nz
  FastDiv div_x;     // division by nx
  FastDiv div_xy;    // division by nx * ny
  double* acc;       // the replica's statistics accumulators (kAccDoubles)
};

struct BatchArgs {
  const ReplicaArgs* __restrict__ reps;  // device table, one entry per replica
  const uint32_t* __restrict__ tile_rep; // replica of each tile
  uint32_t ntiles;                       // tiles of blockDim.x consecutive nodes, all replicas
  const uint32_t* step;                  // device step counter
  uint32_t step_offset;                  // t mod 2^32 = *step + step_offset
  uint32_t partial_pitch;                // doubles between partial columns (>= ntiles)
  double* partials;                      // statistics partials [kNumStats][partial_pitch]
};

// One step of every replica (persistent grid of `grid` blocks walking the tiles);
// the Philox step count is *b.step + b.step_offset, and the parity `odd` must
// match it.  all_ghost_eq: every replica has every omega_g = 1 (then the
// kernel variant without the general ghost relaxation runs).  stats: each
// tile's statistics go to column `tile` of b.partials.
hipError_t launch_batch_step(int storage, bool odd, int rounds, bool all_ghost_eq, bool stats,
                             const BatchArgs& b, uint32_t grid, uint32_t tile, hipStream_t stream);
// Adds each replica's tile partials (tiles of `tile` nodes) into its accumulators.
hipError_t launch_batch_stats_reduce(const BatchArgs& b, uint32_t nrep, uint32_t tile, hipStream_t stream);
// *step += delta on the device (the last node of a captured graph of steps).
hipError_t launch_advance_step(uint32_t* step, uint32_t delta, hipStream_t stream);

// Launch configuration of the step kernel.
struct Launch {
  uint32_t bx, by;   // block shape (bx * by <= 256, bx multiple of 64)
  uint32_t grid;     // number of blocks (ntiles rounded up to a multiple of 8)
};

Launch make_launch(uint32_t nx, uint32_t ny, uint32_t nz, uint32_t bx, uint32_t by);

// One fused stream + collide step on `stream`.  rounds: 0 (no noise), 7 or 10.
hipError_t launch_step(int storage, bool odd, int rounds, bool stats, const StepArgs& a,
                       const Launch& l, hipStream_t stream);

// Even step without statistics in one-wave blocks (nx a multiple of 64).
hipError_t launch_step_wave(int storage, int rounds, const StepArgs& a, hipStream_t stream);

// True when the odd step can run in whole-row blocks: nx a multiple of 64, at
// most 64 kMaxRowWaves.
bool row_kernel_fits(uint32_t nx);
// A step in whole-row blocks, one block per x-row (a.xcd_remap applies to
// rows): odd steps with or without statistics (every store a whole aligned
// cache line), even steps with statistics only.  With stats, one statistics
// partial per block of the row_grid(ny, nz) blocks.
hipError_t launch_step_row(int storage, bool odd, int rounds, bool stats, const StepArgs& a, hipStream_t stream);
// Number of blocks of the whole-row odd step: ny nz rounded up to a multiple of 8.
uint32_t row_grid(uint32_t ny, uint32_t nz);

// Deterministic reduction of the statistics partials into the accumulators.
// scratch holds at least 2 * kNumStats * ceil(grid / 2048) doubles.
hipError_t launch_stats_reduce(const double* partials, uint32_t grid, double* scratch,
                               double* acc, hipStream_t stream);

struct GatherArgs {
  const void* pop;
  uint32_t nx, ny, nz;
  uint64_t pop_pitch;     // elements from population row i to row i + 1 of a block (Q)
  uint64_t row_pitch;     // elements from one x-row block to the next in y inside a brick (R)
  uint64_t ybrick_pitch;  // elements from one brick to the next in y (Yb)
  uint64_t zin_pitch;     // elements from one x-row block to the next in z inside a brick (Zi)
  uint64_t plane_pitch;   // elements from one brick row (Bz z planes) to the next (P)
  uint32_t by_log, bz_log;  // brick shape, as in StepArgs
  uint32_t odd;           // parity of the current step count
  double rho0;
  float sigma[4];
  float inv_sigma[4];
};

// f(x, t) -> dst[i * N + n] (FP64, absolute populations).
hipError_t launch_get_populations(int storage, const GatherArgs& g, double* dst, hipStream_t s);
// f(x, t) at nodes[0..count) -> dst[i * count + k] (FP64, absolute); an index
// >= nx ny nz reads nothing and yields NaN.
hipError_t launch_get_populations_at(int storage, const GatherArgs& g, const uint32_t* nodes,
                                     uint32_t count, double* dst, hipStream_t s);
// src[i * N + n] (FP64, absolute) -> storage slots for step parity g.odd.
hipError_t launch_set_populations(int storage, const GatherArgs& g, const double* src,
                                  hipStream_t s);
// Equilibrium f^(0)(rho, u) (rho, u may be null) -> storage slots.
hipError_t launch_init_equilibrium(int storage, const GatherArgs& g, const double* rho,
                                   const double* u, hipStream_t s);
// f^(0)(rho, u) plus Gaussian deviations of covariance rho0 kT w_i / cs2.
hipError_t launch_init_thermal(int storage, const GatherArgs& g, const double* rho, const double* u,
                               uint32_t key0, uint32_t key1, uint32_t sid, int rounds, double kT,
                               hipStream_t s);
// Moment fields (FP32, planar) selected by mask (1 rho, 2 j, 4 Pi).
hipError_t launch_get_moments(int storage, const GatherArgs& g, uint32_t mask, float* dst,
                              hipStream_t s);
// The same fields for the nodes n0 .. n0 + count - 1 only: field c of node
// n0 + k -> dst[c * pitch + k] (bit for bit the values of launch_get_moments).
hipError_t launch_get_moments_range(int storage, const GatherArgs& g, uint32_t mask, uint64_t n0,
                                    uint64_t count, float* dst, uint64_t pitch, hipStream_t s);
// Re-encodes stored deviations after a change of rho0 or sigma.
hipError_t launch_reencode(int storage, const GatherArgs& from, const GatherArgs& to,
                           hipStream_t s);

hipError_t launch_rng_normals(uint32_t key0, uint32_t key1, uint32_t stream_id, int rounds,
                              uint32_t node0, uint32_t count, uint32_t step, float* u, float* z,
                              hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t launch_fill_zero(double* dst, size_t n, hipStream_t s);
// *dst = value (one thread), stream ordered.
hipError_t launch_set_u32(uint32_t* dst, uint32_t value, hipStream_t s);

}  // namespace rflbm
