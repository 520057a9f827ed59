// lattice.hpp -- internal state of a lattice object and the helpers shared by
// the single-box interface (api.cpp) and the batched one (batch.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cstdint>
#include <string>

#include "../../include/rflbm.h"
#include "kernels.hpp"

namespace rflbm {

// Device buffer of one lattice: the x-row blocked populations, then the instability
// flag, the FP64 accumulators, the statistics partials and reduction scratch.
struct Layout {
  uint32_t pop_pitch;    // bytes between the population rows of one x-row block
  uint32_t row_pitch;    // bytes between x-row blocks (27 population rows) in y inside a brick
  uint32_t ybrick_pitch; // bytes between bricks in y
  uint32_t zin_pitch;    // bytes between x-row blocks in z inside a brick
  uint32_t by_log, bz_log;  // brick shape (kernels.hpp); 0, 0: plain layout
  uint64_t plane_pitch;  // bytes between brick rows (between z planes when bz_log = 0)
  size_t pop_bytes;
  size_t flag_off, acc_off, partial_off, scratch_off, total;
  uint32_t grid_max;
};

constexpr size_t kAlign = 256;

// Padding (bytes) appended to every population row, every x-row block and
// every z plane of the population array.
#ifndef RFLBM_POP_PAD
#define RFLBM_POP_PAD 0
#endif
#ifndef RFLBM_ROW_PAD
#define RFLBM_ROW_PAD 0
#endif
#ifndef RFLBM_PLANE_PAD
#define RFLBM_PLANE_PAD 0
#endif
static_assert(RFLBM_POP_PAD % 128 == 0 && RFLBM_ROW_PAD % 256 == 0 && RFLBM_PLANE_PAD % 256 == 0,
              "pads keep rows aligned to cache lines");

size_t align_up(size_t v, size_t a);
uint64_t node_count(const rflbm_params& p);
std::string validate(const rflbm_params* p);
// Layout of a lattice's buffer; `bricks`: row blocks in bricks where the box
// allows (single boxes), else the plain layout (batch replicas).
Layout layout_for(const rflbm_params& p, bool bricks = true);
uint64_t pop_pitch_of(const rflbm_params& p);    // bytes between population rows
uint64_t row_pitch_of(const rflbm_params& p);    // bytes between x-row blocks
uint64_t plane_pitch_of(const rflbm_params& p);  // bytes between z planes (plain layout)
rflbm_status fail(rflbm_status st, const std::string& msg);

}  // namespace rflbm

struct rflbm_lattice {
  rflbm_params p;
  rflbm::Layout L;
  uint8_t* buf = nullptr;
  bool owns_buf = false;
  bool is_view = false;  // a replica of a batch (borrowed, destroyed with the batch)
  hipStream_t stream = nullptr;
  int device = 0;  // HIP device current when the lattice was set up
  int64_t t = 0;
  int32_t stats_every = 0;
  rflbm::Launch launch{};
  bool xcd_remap = true;
  // row-aligned blocks for steps without statistics (on by default), used
  // where the step is bandwidth bound (FP32 storage, or k_BT = 0): even steps
  // in one-wave x-segments, odd steps in whole-row blocks when nx fits
  bool row_mode = true;
  // S(k) state (library-allocated on first use)
  hipfftHandle plan = 0;
  bool have_plan = false;
  float* sk_fields = nullptr;               // 10 N floats
  void* sk_spec = nullptr;                  // nz ny (nx/2 + 1) complex
  double* sk_sums = nullptr;                // 10 nshells
  unsigned long long* sk_counts = nullptr;  // nshells
  int64_t sk_samples = 0;
  int32_t nshells = 0;
};

namespace rflbm {

// Kernel arguments of one step of lattice L (everything but the step count).
StepArgs step_args(const rflbm_lattice* L);
// Arguments of the readback and set-up kernels for lattice L with parameters p
// at step count t (the parity of t selects the AA layout).
GatherArgs gather_args(const rflbm_lattice* L, const rflbm_params& p, int64_t t);
// Sets up a lattice object on an existing buffer (no allocation, no kernels).
// `bricks` as for layout_for.
void lattice_init(rflbm_lattice* L, const rflbm_params& p, uint8_t* buf, hipStream_t s, bool bricks = true);
// Zeroes the populations (rest state), flag and accumulators of L.
hipError_t lattice_clear(rflbm_lattice* L);
// Releases what the library allocated for L (S(k) scratch, owned buffer).
void lattice_release(rflbm_lattice* L);
// The single-lattice operations without the checks that keep batch replicas
// consistent (the batch calls these for its replicas).
rflbm_status lattice_steps(rflbm_lattice* L, int64_t nsteps);
rflbm_status lattice_set_params(rflbm_lattice* L, const rflbm_params* p);
rflbm_status lattice_set_step_count(rflbm_lattice* L, int64_t t);
// Bytes of scratch a change of parity of L needs (one population plane).
size_t parity_scratch_bytes(const rflbm_lattice* L);
// lattice_set_step_count with the caller's scratch (at least
// parity_scratch_bytes(L) bytes of device memory; unused if the parity stays).
rflbm_status lattice_set_step_count_with(rflbm_lattice* L, int64_t t, void* tmp);

}  // namespace rflbm

namespace rflbm {
// Reports a failed HIP call.  HIP keeps the error as the thread's last error,
// which the launch wrappers read back after every launch; it is cleared here
// so that a later, unrelated call does not report it again.
inline rflbm_status hip_fail(rflbm_status st, const std::string& what, hipError_t e) {
  (void)hipGetLastError();
  return fail(st, what + ": " + hipGetErrorString(e));
}
}  // namespace rflbm

#define RFLBM_HIP(call)                                                  \
  do {                                                                   \
    const hipError_t e_ = (call);                                        \
    if (e_ != hipSuccess) return ::rflbm::hip_fail(RFLBM_EHIP, #call, e_); \
  } while (0)
