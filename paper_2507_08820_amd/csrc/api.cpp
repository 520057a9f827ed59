// api.cpp -- implementation of the C interface declared in include/rflbm.h: a
// lattice object owning (or borrowing) one device buffer, the derivation of the
// per-mode relaxation factors and noise amplitudes of Eq. fluct_phi, step
// sequencing (AA parity, Philox step counter, statistics), and readback.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/rflbm.h"
#include "d3q27.hpp"
#include "kernels.hpp"
#include "lattice.hpp"
#include "storage.hpp"

namespace rflbm {
hipError_t launch_sk_bin(const void* spec, uint32_t nx, uint32_t ny, uint32_t nz, uint32_t nshells,
                         double* shell_sum, unsigned long long* shell_count, hipStream_t s);
// Moves the stored state to the other AA parity in place, as raw stored words;
// tmp holds one population plane (nx ny nz words of the storage type).
hipError_t launch_swap_parity(int storage, const GatherArgs& g, void* tmp, hipStream_t s);
}

using namespace rflbm;

namespace {

thread_local std::string g_last_error;

constexpr double kCs2 = 1.0 / 3.0;
// Supported block shapes of the step kernel: (bx, 256 / bx).
constexpr uint32_t kBlockX[3] = {64, 128, 256};

bool valid_tau(double t) { return std::isfinite(t) && t > 0.5; }

double fdt(double omega) { return std::sqrt(omega * (2.0 - omega)); }

}  // namespace

namespace rflbm {

rflbm_status fail(rflbm_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

uint64_t node_count(const rflbm_params& p) {
  return static_cast<uint64_t>(p.nx) * static_cast<uint64_t>(p.ny) * static_cast<uint64_t>(p.nz);
}

std::string validate(const rflbm_params* p) {
  if (!p) return "params is NULL";
  if (p->nx < 2 || p->ny < 2 || p->nz < 2) return "box dimensions must each be >= 2";
  if (p->storage < RFLBM_F32 || p->storage > RFLBM_BF16) return "unknown storage type";
  if (p->model != RFLBM_MODEL_REG && p->model != RFLBM_MODEL_BGK && p->model != RFLBM_MODEL_REC)
    return "unknown model";
  if (p->philox_rounds != 7 && p->philox_rounds != 10) return "philox_rounds must be 7 or 10";
  if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) return "rho0 must be positive";
  if (!(p->kT >= 0.0) || !std::isfinite(p->kT)) return "kT must be >= 0";
  if (!valid_tau(p->tau_shear) || !valid_tau(p->tau_bulk))
    return "tau_shear and tau_bulk must exceed 1/2 (omega (2 - omega) > 0 in Eq. fluct_phi)";
  for (int k = 0; k < 17; ++k)
    if (!valid_tau(p->tau_ghost[k])) return "every tau_ghost must exceed 1/2";
  if (p->reserved != 0) return "reserved must be 0";
  if (!(p->storage_scale >= 0.0) || !std::isfinite(p->storage_scale)) return "storage_scale must be >= 0";
  if (p->storage != RFLBM_F32 && p->storage_scale == 0.0 && p->kT == 0.0)
    return "16-bit storage with kT = 0 needs a storage_scale";
  const uint64_t n = node_count(*p);
  if (n >= (1ull << 32)) return "box has 2^32 or more nodes";
  if (static_cast<uint64_t>(p->ny) * row_pitch_of(*p) >= (1ull << 32))
    return "one z plane of populations (27 nx ny values) must stay below 4 GiB";
  return "";
}

uint64_t pop_pitch_of(const rflbm_params& p) {
  return static_cast<uint64_t>(p.nx) * storage_bytes(p.storage) + RFLBM_POP_PAD;
}

uint64_t row_pitch_of(const rflbm_params& p) { return 27ull * pop_pitch_of(p) + RFLBM_ROW_PAD; }

uint64_t plane_pitch_of(const rflbm_params& p) {
  return static_cast<uint64_t>(p.ny) * row_pitch_of(p) + RFLBM_PLANE_PAD;
}

// Brick shape of the row blocks, log2 (kernels.hpp): 2 rows x 16 planes, each
// side halved until it divides the box, and the planes halved until one brick
// row (ny rows of Bz planes) stays below 4 GiB, the reach of the kernels'
// 32-bit lane offsets.  Measured on the odd step's access pattern at 512^3 FP32
// (27 loads from the 9 row blocks around a row, 27 stores to them, rows in
// memory order): plain layout 5.36 ms; bricks of 2 x 16 5.02 ms, 2 x 8 5.05,
// 1 x 16 5.08, 8 x 8 5.09, 2 x 4 and 4 x 8 5.11-5.12, 2 x 32 5.15.  The even
// step, a sequential walk in either layout, is unchanged (4.73 ms).
constexpr uint32_t kBrickYLog = 1, kBrickZLog = 4;

static void brick_shape(const rflbm_params& p, uint32_t& by_log, uint32_t& bz_log) {
  by_log = kBrickYLog;
  while (by_log > 0 && p.ny % (1 << by_log) != 0) --by_log;
  bz_log = kBrickZLog;
  while (bz_log > 0 && (p.nz % (1 << bz_log) != 0 ||
                        (static_cast<uint64_t>(p.ny) << bz_log) * row_pitch_of(p) >= (1ull << 32)))
    --bz_log;
}

Layout layout_for(const rflbm_params& p, bool bricks) {
  Layout L;
  L.pop_pitch = static_cast<uint32_t>(pop_pitch_of(p));
  L.row_pitch = static_cast<uint32_t>(row_pitch_of(p));
  L.by_log = L.bz_log = 0;
  if (bricks) brick_shape(p, L.by_log, L.bz_log);
  L.zin_pitch = L.row_pitch << L.by_log;
  L.ybrick_pitch = L.zin_pitch << L.bz_log;
  // a brick row: ny / By bricks, plus the plane padding (plain layout: one plane)
  L.plane_pitch = static_cast<uint64_t>(p.ny >> L.by_log) * L.ybrick_pitch + RFLBM_PLANE_PAD;
  L.pop_bytes = align_up(static_cast<size_t>(p.nz >> L.bz_log) * L.plane_pitch, kAlign);
  L.grid_max = 0;
  for (uint32_t bx : kBlockX) {
    const Launch l = make_launch(p.nx, p.ny, p.nz, bx, 256 / bx);
    if (l.grid > L.grid_max) L.grid_max = l.grid;
  }
  L.flag_off = L.pop_bytes;
  L.acc_off = L.flag_off + kAlign;
  L.partial_off = L.acc_off + align_up(kAccDoubles * sizeof(double), kAlign);
  L.scratch_off = L.partial_off + align_up(static_cast<size_t>(kNumStats) * L.grid_max * sizeof(double), kAlign);
  const size_t chunks = (L.grid_max + 2047) / 2048;
  L.total = L.scratch_off + align_up(2 * static_cast<size_t>(kNumStats) * chunks * sizeof(double), kAlign);
  return L;
}

}  // namespace rflbm

namespace {

uint64_t nodes(const rflbm_lattice* L) { return node_count(L->p); }

void sigma_of(const rflbm_params& p, float sigma[4], float inv[4]) {
  double scale = 1.0;
  if (p.storage != RFLBM_F32) scale = p.storage_scale > 0.0 ? p.storage_scale : std::sqrt(p.rho0 * p.kT / kCs2);
  for (int c = 0; c < 4; ++c) {
    const double s = p.storage == RFLBM_F32 ? 1.0 : std::sqrt(class_weight(c)) * scale;
    sigma[c] = static_cast<float>(s);
    inv[c] = static_cast<float>(1.0 / s);
  }
}

}  // namespace

namespace rflbm {

GatherArgs gather_args(const rflbm_lattice* L, const rflbm_params& p, int64_t t) {
  GatherArgs g;
  g.pop = L->buf;
  g.nx = p.nx;
  g.ny = p.ny;
  g.nz = p.nz;
  g.pop_pitch = L->L.pop_pitch / storage_bytes(p.storage);
  g.row_pitch = L->L.row_pitch / storage_bytes(p.storage);
  g.ybrick_pitch = L->L.ybrick_pitch / storage_bytes(p.storage);
  g.zin_pitch = L->L.zin_pitch / storage_bytes(p.storage);
  g.plane_pitch = L->L.plane_pitch / storage_bytes(p.storage);
  g.by_log = L->L.by_log;
  g.bz_log = L->L.bz_log;
  g.odd = static_cast<uint32_t>(t & 1);
  g.rho0 = p.rho0;
  sigma_of(p, g.sigma, g.inv_sigma);
  return g;
}

}  // namespace rflbm

namespace rflbm {

StepArgs step_args(const rflbm_lattice* L) {
  const rflbm_params& p = L->p;
  StepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.pop = L->buf;
  a.nx = p.nx;
  a.ny = p.ny;
  a.nz = p.nz;
  a.pop_pitch = L->L.pop_pitch;
  a.row_pitch = L->L.row_pitch;
  a.ybrick_pitch = L->L.ybrick_pitch;
  a.zin_pitch = L->L.zin_pitch;
  a.by_log = L->L.by_log;
  a.bz_log = L->L.bz_log;
  a.plane_pitch = L->L.plane_pitch;
  a.tiles_x = (p.nx + L->launch.bx - 1) / L->launch.bx;
  a.tiles_y = (p.ny + L->launch.by - 1) / L->launch.by;
  a.ntiles = a.tiles_x * a.tiles_y * static_cast<uint32_t>(p.nz);
  const auto fd = [](uint32_t d) { return d >= 2 ? make_fastdiv(d) : FastDiv{0u, 1u}; };
  a.div_tiles_x = fd(a.tiles_x);
  a.div_tiles_y = fd(a.tiles_y);
  a.div_ny = fd(static_cast<uint32_t>(p.ny));
  a.div_nyb = fd(static_cast<uint32_t>(p.ny) >> L->L.by_log);
  a.div_segs = fd(static_cast<uint32_t>(p.nx) / 64u);
  a.xcd_remap = L->xcd_remap ? 1u : 0u;
  a.key0 = static_cast<uint32_t>(p.seed & 0xffffffffu);
  a.key1 = static_cast<uint32_t>(p.seed >> 32);
  a.stream_id = p.stream_id;
  a.rho0 = static_cast<float>(p.rho0);
  const bool bgk = p.model == RFLBM_MODEL_BGK;
  const double om_s = 1.0 / p.tau_shear;
  const double om_b = bgk ? om_s : 1.0 / p.tau_bulk;
  a.lam_s = static_cast<float>(1.0 - om_s);
  a.lam_b_minus_s = static_cast<float>((1.0 - om_b) - (1.0 - om_s));
  // phi_k = sqrt(rho) sqrt(kT b_k / cs2) sqrt(omega_k (2 - omega_k))  (Eq. fluct_phi)
  const double kt = p.kT;
  const double base4 = std::sqrt(kt * mode_norm(4) / kCs2);
  // the step kernels carry mode k pre-multiplied by inv_scale of its register
  // slot (the scaled inverse transform), so its noise amplitude carries it too
  // (xx, yy, zz share one scale, as do xy, xz, yz)
  a.amp_s = static_cast<float>(inv_scale(mode_slot(4)) * base4 * fdt(om_s));
  a.amp_b_minus_s = static_cast<float>(inv_scale(mode_slot(4)) * base4 * (fdt(om_b) - fdt(om_s)));
  a.amp_off = static_cast<float>(inv_scale(mode_slot(7)) * std::sqrt(kt * mode_norm(7) / kCs2) * fdt(om_s));
  for (int k = 10; k < 27; ++k) {
    const double om_g = bgk ? om_s : 1.0 / p.tau_ghost[k - 10];
    a.lam_g[k - 10] = static_cast<float>(1.0 - om_g);
    a.amp_g[k - 10] =
        static_cast<float>(inv_scale(mode_slot(k)) * std::sqrt(kt * mode_norm(k) / kCs2) * fdt(om_g));
  }
  a.ghost_eq = 1;
  for (int k = 0; k < 17; ++k)
    if (a.lam_g[k] != 0.0f) a.ghost_eq = 0;
  // at omega_g = 1 the relaxed ghost part vanishes in either reading
  a.ghost_rec = (p.model == RFLBM_MODEL_REC && !a.ghost_eq) ? 1u : 0u;
  sigma_of(p, a.sigma, a.inv_sigma);
  a.flag = reinterpret_cast<int*>(L->buf + L->L.flag_off);
  a.partials = reinterpret_cast<double*>(L->buf + L->L.partial_off);
  return a;
}

void lattice_init(rflbm_lattice* L, const rflbm_params& p, uint8_t* buf, hipStream_t s, bool bricks) {
  L->p = p;
  L->L = layout_for(p, bricks);
  L->buf = buf;
  L->stream = s;
  if (hipGetDevice(&L->device) != hipSuccess) {
    (void)hipGetLastError();
    L->device = 0;
  }
  L->launch = make_launch(p.nx, p.ny, p.nz, p.nx >= 256 ? 256 : (p.nx >= 128 ? 128 : 64),
                          p.nx >= 256 ? 1 : (p.nx >= 128 ? 2 : 4));
  L->row_mode = true;
}

// Row-aligned blocks pay off where the step is bandwidth bound: FP32 storage,
// or no noise (16-bit at 512^3 without noise: 2.46 ms per step against 2.74 ms
// tiled).  The 16-bit steps with noise are bound by arithmetic: there the lane
// moves and barriers of the whole-row odd step cost more than the aligned
// accesses save (3.8 against 3.2 ms), and one-wave even steps between tiled
// odd ones measured no faster than tiled ones (3.28-3.30 against 3.26-3.27 ms
// per step), so those steps keep the tiled kernel.
static bool rows_pay(const rflbm_lattice* L) {
  return L->row_mode && (L->p.storage == RFLBM_F32 || L->p.kT == 0.0);
}

static bool odd_in_rows(const rflbm_lattice* L) { return rows_pay(L) && row_kernel_fits(L->p.nx); }

hipError_t lattice_clear(rflbm_lattice* L) {
  // populations (deviation 0 = rest at rho0), flag and accumulators
  return hipMemsetAsync(L->buf, 0, L->L.scratch_off, L->stream);
}

void lattice_release(rflbm_lattice* L) {
  if (L->have_plan) (void)hipfftDestroy(L->plan);
  if (L->sk_fields) (void)hipFree(L->sk_fields);
  if (L->sk_spec) (void)hipFree(L->sk_spec);
  if (L->sk_sums) (void)hipFree(L->sk_sums);
  if (L->sk_counts) (void)hipFree(L->sk_counts);
  if (L->owns_buf) (void)hipFree(L->buf);
  L->have_plan = false;
  L->sk_fields = nullptr;
  L->sk_spec = nullptr;
  L->sk_sums = nullptr;
  L->sk_counts = nullptr;
  L->buf = nullptr;
}

}  // namespace rflbm

namespace {

rflbm_status check_lattice(const rflbm_lattice* L) {
  if (!L) return fail(RFLBM_EINVAL, "lattice is NULL");
  return RFLBM_OK;
}

rflbm_status clear_flag(rflbm_lattice* L) {
  RFLBM_HIP(launch_fill_zero(reinterpret_cast<double*>(L->buf + L->L.flag_off), 1, L->stream));
  return RFLBM_OK;
}

// Copies a host array to a temporary device buffer (or passes a device pointer through).
struct DeviceIn {
  const void* ptr = nullptr;
  void* owned = nullptr;
  ~DeviceIn() {
    if (owned) (void)hipFree(owned);
  }
};

rflbm_status stage_in(const void* src, size_t bytes, bool is_host, hipStream_t s, DeviceIn& out) {
  if (!src) return RFLBM_OK;
  if (!is_host) {
    out.ptr = src;
    return RFLBM_OK;
  }
  RFLBM_HIP(hipMalloc(&out.owned, bytes));
  RFLBM_HIP(hipMemcpyAsync(out.owned, src, bytes, hipMemcpyHostToDevice, s));
  RFLBM_HIP(hipStreamSynchronize(s));
  out.ptr = out.owned;
  return RFLBM_OK;
}

}  // namespace

namespace rflbm {

rflbm_status lattice_set_params(rflbm_lattice* L, const rflbm_params* p) {
  const std::string err = validate(p);
  if (!err.empty()) return fail(RFLBM_EINVAL, err);
  if (p->nx != L->p.nx || p->ny != L->p.ny || p->nz != L->p.nz || p->storage != L->p.storage)
    return fail(RFLBM_EINVAL, "box size and storage type are fixed at creation");
  const GatherArgs from = gather_args(L, L->p, L->t);
  const GatherArgs to = gather_args(L, *p, L->t);
  const bool reencode = from.rho0 != to.rho0 || std::memcmp(from.sigma, to.sigma, sizeof(from.sigma)) != 0;
  if (reencode) RFLBM_HIP(launch_reencode(L->p.storage, from, to, L->stream));
  L->p = *p;
  return RFLBM_OK;
}

rflbm_status lattice_steps(rflbm_lattice* L, int64_t nsteps) {
  if (nsteps < 0) return fail(RFLBM_EINVAL, "nsteps must be >= 0");
  StepArgs a = step_args(L);
  const int rounds = L->p.kT > 0.0 ? static_cast<int>(L->p.philox_rounds) : 0;
  double* acc = reinterpret_cast<double*>(L->buf + L->L.acc_off);
  double* scratch = reinterpret_cast<double*>(L->buf + L->L.scratch_off);
  for (int64_t s = 0; s < nsteps; ++s) {
    const int64_t t = L->t;
    const bool stats = L->stats_every > 0 && (t % L->stats_every) == 0;
    a.step = static_cast<uint32_t>(t & 0xffffffffu);
    const bool odd = (t & 1) != 0;
    uint32_t grid = L->launch.grid;  // blocks, hence statistics partials, of the kernel used
    if ((odd || stats) && odd_in_rows(L)) {
      // whole rows: odd steps, and even steps with statistics (one partial per
      // row; the one-wave even blocks would write one per wave)
      RFLBM_HIP(launch_step_row(L->p.storage, odd, rounds, stats, a, L->stream));
      grid = row_grid(L->p.ny, L->p.nz);
    } else if (!odd && !stats && rows_pay(L) && L->p.nx % 64 == 0) {
      RFLBM_HIP(launch_step_wave(L->p.storage, rounds, a, L->stream));
    } else {
      RFLBM_HIP(launch_step(L->p.storage, odd, rounds, stats, a, L->launch, L->stream));
    }
    if (stats) RFLBM_HIP(launch_stats_reduce(a.partials, grid, scratch, acc, L->stream));
    L->t = t + 1;
  }
  return RFLBM_OK;
}

size_t parity_scratch_bytes(const rflbm_lattice* L) { return nodes(L) * storage_bytes(L->p.storage); }

rflbm_status lattice_set_step_count_with(rflbm_lattice* L, int64_t t, void* tmp) {
  if (t < 0) return fail(RFLBM_EINVAL, "step count must be >= 0");
  if ((t & 1) != (L->t & 1)) {
    // the storage layout depends on the parity: move the state to the new one,
    // in place and bit for bit, through one population plane of scratch
    hipError_t e = launch_swap_parity(L->p.storage, gather_args(L, L->p, L->t), tmp, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) return hip_fail(RFLBM_EHIP, "re-layout", e);
  }
  L->t = t;
  return RFLBM_OK;
}

rflbm_status lattice_set_step_count(rflbm_lattice* L, int64_t t) {
  if (t < 0) return fail(RFLBM_EINVAL, "step count must be >= 0");
  void* tmp = nullptr;
  if ((t & 1) != (L->t & 1)) {
    if (const hipError_t m = hipMalloc(&tmp, parity_scratch_bytes(L)); m != hipSuccess)
      return hip_fail(RFLBM_ENOMEM, "re-layout scratch", m);
  }
  const rflbm_status st = lattice_set_step_count_with(L, t, tmp);
  if (tmp) (void)hipFree(tmp);
  return st;
}

}  // namespace rflbm

extern "C" {

void rflbm_params_default(rflbm_params* p, int32_t nx, int32_t ny, int32_t nz) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->nx = nx;
  p->ny = ny;
  p->nz = nz;
  p->storage = RFLBM_F32;
  p->model = RFLBM_MODEL_REG;
  p->philox_rounds = 7;
  p->rho0 = 1.0;
  p->kT = 0.0;
  p->tau_shear = 1.0;
  p->tau_bulk = 1.0;
  for (int k = 0; k < 17; ++k) p->tau_ghost[k] = 1.0;
  p->seed = 1;
  p->stream_id = 0;
  p->storage_scale = 0.0;
}

size_t rflbm_required_bytes(const rflbm_params* p) {
  if (!validate(p).empty()) return 0;
  return layout_for(*p).total;
}

rflbm_status rflbm_create(const rflbm_params* p, void* dev_buf, size_t bytes, void* hip_stream,
                          rflbm_lattice** out) {
  if (!out) return fail(RFLBM_EINVAL, "out is NULL");
  *out = nullptr;
  const std::string err = validate(p);
  if (!err.empty()) return fail(RFLBM_EINVAL, err);
  const Layout lay = layout_for(*p);
  if (dev_buf && bytes < lay.total)
    return fail(RFLBM_ENOMEM, "caller buffer smaller than rflbm_required_bytes");
  if (dev_buf && (reinterpret_cast<uintptr_t>(dev_buf) % kAlign) != 0)
    return fail(RFLBM_EINVAL, "caller buffer must be 256-byte aligned");
  rflbm_lattice* L = new (std::nothrow) rflbm_lattice();
  if (!L) return fail(RFLBM_ENOMEM, "host allocation failed");
  uint8_t* buf = static_cast<uint8_t*>(dev_buf);
  if (!buf) {
    void* b = nullptr;
    const hipError_t e = hipMalloc(&b, lay.total);
    if (e != hipSuccess) {
      delete L;
      return hip_fail(RFLBM_ENOMEM, "hipMalloc", e);
    }
    buf = static_cast<uint8_t*>(b);
    L->owns_buf = true;
  }
  lattice_init(L, *p, buf, static_cast<hipStream_t>(hip_stream));
  const hipError_t e = lattice_clear(L);
  if (e != hipSuccess) {
    lattice_release(L);
    delete L;
    return hip_fail(RFLBM_EHIP, "hipMemsetAsync", e);
  }
  *out = L;
  return RFLBM_OK;
}

rflbm_status rflbm_destroy(rflbm_lattice* L) {
  if (!L) return RFLBM_OK;
  if (L->is_view) return fail(RFLBM_ESTATE, "a replica view is released with its batch");
  (void)hipStreamSynchronize(L->stream);
  lattice_release(L);
  delete L;
  return RFLBM_OK;
}

rflbm_status rflbm_set_params(rflbm_lattice* L, const rflbm_params* p) {
  if (rflbm_status s = check_lattice(L)) return s;
  if (L->is_view) return fail(RFLBM_ESTATE, "replicas of a batch change parameters with rflbm_batch_set_params");
  return lattice_set_params(L, p);
}



rflbm_status rflbm_get_params(const rflbm_lattice* L, rflbm_params* p) {
  if (rflbm_status s = check_lattice(L)) return s;
  if (!p) return fail(RFLBM_EINVAL, "params is NULL");
  *p = L->p;
  return RFLBM_OK;
}

rflbm_status rflbm_init_equilibrium(rflbm_lattice* L, const double* rho, const double* u, int host_ptrs) {
  if (rflbm_status s = check_lattice(L)) return s;
  const uint64_t N = nodes(L);
  DeviceIn drho, du;
  if (rflbm_status s = stage_in(rho, N * sizeof(double), host_ptrs, L->stream, drho)) return s;
  if (rflbm_status s = stage_in(u, 3 * N * sizeof(double), host_ptrs, L->stream, du)) return s;
  RFLBM_HIP(launch_init_equilibrium(L->p.storage, gather_args(L, L->p, L->t),
                                    static_cast<const double*>(drho.ptr), static_cast<const double*>(du.ptr),
                                    L->stream));
  if (rflbm_status s = clear_flag(L)) return s;
  if (host_ptrs) RFLBM_HIP(hipStreamSynchronize(L->stream));
  return RFLBM_OK;
}



rflbm_status rflbm_init_thermal(rflbm_lattice* L, const double* rho, const double* u, int host_ptrs) {
  if (rflbm_status s = check_lattice(L)) return s;
  const uint64_t N = nodes(L);
  DeviceIn drho, du;
  if (rflbm_status s = stage_in(rho, N * sizeof(double), host_ptrs, L->stream, drho)) return s;
  if (rflbm_status s = stage_in(u, 3 * N * sizeof(double), host_ptrs, L->stream, du)) return s;
  RFLBM_HIP(launch_init_thermal(L->p.storage, gather_args(L, L->p, L->t), static_cast<const double*>(drho.ptr),
                                static_cast<const double*>(du.ptr), static_cast<uint32_t>(L->p.seed & 0xffffffffu),
                                static_cast<uint32_t>(L->p.seed >> 32), L->p.stream_id,
                                static_cast<int>(L->p.philox_rounds), L->p.kT, L->stream));
  if (rflbm_status s = clear_flag(L)) return s;
  if (host_ptrs) RFLBM_HIP(hipStreamSynchronize(L->stream));
  return RFLBM_OK;
}

rflbm_status rflbm_step(rflbm_lattice* L, int64_t nsteps) {
  if (rflbm_status s = check_lattice(L)) return s;
  if (L->is_view) return fail(RFLBM_ESTATE, "replicas of a batch are stepped with rflbm_batch_step");
  return lattice_steps(L, nsteps);
}

rflbm_status rflbm_sync(rflbm_lattice* L) {
  if (rflbm_status s = check_lattice(L)) return s;
  int flag = 0;
  RFLBM_HIP(hipMemcpyAsync(&flag, L->buf + L->L.flag_off, sizeof(int), hipMemcpyDeviceToHost, L->stream));
  RFLBM_HIP(hipStreamSynchronize(L->stream));
  if (flag) return fail(RFLBM_EUNSTABLE, "a node reached rho <= 0 or a non-finite density or momentum");
  return RFLBM_OK;
}

int64_t rflbm_step_count(const rflbm_lattice* L) { return L ? L->t : -1; }

rflbm_status rflbm_set_step_count(rflbm_lattice* L, int64_t t) {
  if (rflbm_status s = check_lattice(L)) return s;
  if (L->is_view) return fail(RFLBM_ESTATE, "replicas of a batch share the batch's step count");
  return lattice_set_step_count(L, t);
}



rflbm_status rflbm_get_populations(rflbm_lattice* L, double* dst, int dst_is_host) {
  if (rflbm_status s = check_lattice(L)) return s;
  if (!dst) return fail(RFLBM_EINVAL, "dst is NULL");
  const uint64_t N = nodes(L);
  const GatherArgs g = gather_args(L, L->p, L->t);
  if (!dst_is_host) {
    RFLBM_HIP(launch_get_populations(L->p.storage, g, dst, L->stream));
    return RFLBM_OK;
  }
  double* tmp = nullptr;
  RFLBM_HIP(hipMalloc(&tmp, 27 * N * sizeof(double)));
  hipError_t e = launch_get_populations(L->p.storage, g, tmp, L->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dst, tmp, 27 * N * sizeof(double), hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  (void)hipFree(tmp);
  if (e != hipSuccess) return hip_fail(RFLBM_EHIP, "get_populations", e);
  return RFLBM_OK;
}

rflbm_status rflbm_get_populations_at(rflbm_lattice* L, const uint32_t* nodes, uint32_t count, double* dst) {
  if (rflbm_status s = check_lattice(L)) return s;
  if (count > 0 && (!nodes || !dst)) return fail(RFLBM_EINVAL, "nodes and dst must be device arrays");
  RFLBM_HIP(launch_get_populations_at(L->p.storage, gather_args(L, L->p, L->t), nodes, count, dst, L->stream));
  return RFLBM_OK;
}

rflbm_status rflbm_set_populations(rflbm_lattice* L, const double* src, int src_is_host) {
  if (rflbm_status s = check_lattice(L)) return s;
  if (!src) return fail(RFLBM_EINVAL, "src is NULL");
  const uint64_t N = nodes(L);
  DeviceIn d;
  if (rflbm_status s = stage_in(src, 27 * N * sizeof(double), src_is_host, L->stream, d)) return s;
  RFLBM_HIP(launch_set_populations(L->p.storage, gather_args(L, L->p, L->t), static_cast<const double*>(d.ptr),
                                   L->stream));
  if (rflbm_status s = clear_flag(L)) return s;
  if (src_is_host) RFLBM_HIP(hipStreamSynchronize(L->stream));
  return RFLBM_OK;
}

rflbm_status rflbm_get_moments(rflbm_lattice* L, uint32_t mask, float* dst, int dst_is_host) {
  if (rflbm_status s = check_lattice(L)) return s;
  if (!dst) return fail(RFLBM_EINVAL, "dst is NULL");
  if (mask == 0 || (mask & ~7u)) return fail(RFLBM_EINVAL, "mask must select RHO, J and/or PI");
  const uint64_t N = nodes(L);
  const int nf = ((mask & 1u) ? 1 : 0) + ((mask & 2u) ? 3 : 0) + ((mask & 4u) ? 6 : 0);
  const GatherArgs g = gather_args(L, L->p, L->t);
  if (!dst_is_host) {
    RFLBM_HIP(launch_get_moments(L->p.storage, g, mask, dst, L->stream));
    return RFLBM_OK;
  }
  float* tmp = nullptr;
  RFLBM_HIP(hipMalloc(&tmp, nf * N * sizeof(float)));
  hipError_t e = launch_get_moments(L->p.storage, g, mask, tmp, L->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dst, tmp, nf * N * sizeof(float), hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  (void)hipFree(tmp);
  if (e != hipSuccess) return hip_fail(RFLBM_EHIP, "get_moments", e);
  return RFLBM_OK;
}

rflbm_status rflbm_stats_config(rflbm_lattice* L, int32_t every) {
  if (rflbm_status s = check_lattice(L)) return s;
  if (L->is_view)
    return fail(RFLBM_ESTATE, "statistics of batch replicas are configured with rflbm_batch_stats_config");
  if (every < 0) return fail(RFLBM_EINVAL, "every must be >= 0");
  L->stats_every = every;
  return RFLBM_OK;
}

rflbm_status rflbm_get_stats(rflbm_lattice* L, rflbm_stats* out) {
  if (rflbm_status s = check_lattice(L)) return s;
  if (!out) return fail(RFLBM_EINVAL, "out is NULL");
  double acc[kAccDoubles];
  RFLBM_HIP(hipMemcpyAsync(acc, L->buf + L->L.acc_off, sizeof(acc), hipMemcpyDeviceToHost, L->stream));
  RFLBM_HIP(hipStreamSynchronize(L->stream));
  std::memset(out, 0, sizeof(*out));
  out->samples = static_cast<int64_t>(acc[kNumStats]);
  out->nodes = static_cast<int64_t>(nodes(L));
  out->sum_drho = acc[0];
  out->sum_drho2 = acc[1];
  for (int a = 0; a < 3; ++a) {
    out->sum_j[a] = acc[2 + a];
    out->sum_j2[a] = acc[5 + a];
    out->sum_u2[a] = acc[8 + a];
    out->momentum[a] = acc[kNumStats + 2 + a];
  }
  for (int c = 0; c < 6; ++c) {
    out->sum_pi[c] = acc[11 + c];
    out->sum_pi2[c] = acc[17 + c];
  }
  out->mass_dev = acc[kNumStats + 1];
  return RFLBM_OK;
}

rflbm_status rflbm_reset_stats(rflbm_lattice* L) {
  if (rflbm_status s = check_lattice(L)) return s;
  RFLBM_HIP(launch_fill_zero(reinterpret_cast<double*>(L->buf + L->L.acc_off), kAccDoubles, L->stream));
  return RFLBM_OK;
}

int32_t rflbm_sk_nshells(const rflbm_lattice* L) {
  if (!L) return 0;
  const double h = std::sqrt(std::pow(L->p.nx / 2, 2.0) + std::pow(L->p.ny / 2, 2.0) + std::pow(L->p.nz / 2, 2.0));
  return static_cast<int32_t>(std::llround(h)) + 1;
}

static rflbm_status sk_prepare(rflbm_lattice* L) {
  if (L->have_plan) return RFLBM_OK;
  const uint64_t N = nodes(L);
  L->nshells = rflbm_sk_nshells(L);
  const size_t spec_bytes = static_cast<size_t>(L->p.nx / 2 + 1) * L->p.ny * L->p.nz * 2 * sizeof(float);
  // buffers that an earlier, failed attempt allocated are kept and reused
  if (!L->sk_fields) RFLBM_HIP(hipMalloc(reinterpret_cast<void**>(&L->sk_fields), 10 * N * sizeof(float)));
  if (!L->sk_spec) RFLBM_HIP(hipMalloc(&L->sk_spec, spec_bytes));
  if (!L->sk_sums) RFLBM_HIP(hipMalloc(reinterpret_cast<void**>(&L->sk_sums), 10 * L->nshells * sizeof(double)));
  if (!L->sk_counts)
    RFLBM_HIP(hipMalloc(reinterpret_cast<void**>(&L->sk_counts), L->nshells * sizeof(unsigned long long)));
  RFLBM_HIP(hipMemsetAsync(L->sk_sums, 0, 10 * L->nshells * sizeof(double), L->stream));
  RFLBM_HIP(hipMemsetAsync(L->sk_counts, 0, L->nshells * sizeof(unsigned long long), L->stream));
  hipfftHandle plan;
  if (hipfftPlan3d(&plan, L->p.nz, L->p.ny, L->p.nx, HIPFFT_R2C) != HIPFFT_SUCCESS)
    return fail(RFLBM_EHIP, "hipfftPlan3d failed");
  // the plan is kept only once it runs on the lattice stream
  if (hipfftSetStream(plan, L->stream) != HIPFFT_SUCCESS) {
    (void)hipfftDestroy(plan);
    return fail(RFLBM_EHIP, "hipfftSetStream failed");
  }
  L->plan = plan;
  L->have_plan = true;
  L->sk_samples = 0;
  return RFLBM_OK;
}

rflbm_status rflbm_sk_sample(rflbm_lattice* L) {
  if (rflbm_status s = check_lattice(L)) return s;
  if (rflbm_status s = sk_prepare(L)) return s;
  const uint64_t N = nodes(L);
  RFLBM_HIP(launch_get_moments(L->p.storage, gather_args(L, L->p, L->t), 7u, L->sk_fields, L->stream));
  for (int f = 0; f < 10; ++f) {
    if (hipfftExecR2C(L->plan, L->sk_fields + f * N, static_cast<hipfftComplex*>(L->sk_spec)) != HIPFFT_SUCCESS)
      return fail(RFLBM_EHIP, "hipfftExecR2C failed");
    RFLBM_HIP(launch_sk_bin(L->sk_spec, L->p.nx, L->p.ny, L->p.nz, L->nshells, L->sk_sums + f * L->nshells,
                            (L->sk_samples == 0 && f == 0) ? L->sk_counts : nullptr, L->stream));
  }
  L->sk_samples += 1;
  return RFLBM_OK;
}

rflbm_status rflbm_get_sk(rflbm_lattice* L, int32_t field, double* shell_sum, int64_t* shell_count,
                          int32_t nshells, int64_t* samples) {
  if (rflbm_status s = check_lattice(L)) return s;
  if (field < 0 || field >= 10) return fail(RFLBM_EINVAL, "field must be 0..9");
  if (nshells != rflbm_sk_nshells(L)) return fail(RFLBM_EINVAL, "nshells must equal rflbm_sk_nshells");
  if (samples) *samples = L->sk_samples;
  if (!L->have_plan || L->sk_samples == 0) {
    if (shell_sum) std::memset(shell_sum, 0, nshells * sizeof(double));
    if (shell_count) std::memset(shell_count, 0, nshells * sizeof(int64_t));
    return RFLBM_OK;
  }
  if (shell_sum)
    RFLBM_HIP(hipMemcpyAsync(shell_sum, L->sk_sums + field * L->nshells, nshells * sizeof(double),
                             hipMemcpyDeviceToHost, L->stream));
  if (shell_count)
    RFLBM_HIP(hipMemcpyAsync(shell_count, L->sk_counts, nshells * sizeof(int64_t), hipMemcpyDeviceToHost,
                             L->stream));
  RFLBM_HIP(hipStreamSynchronize(L->stream));
  return RFLBM_OK;
}

rflbm_status rflbm_reset_sk(rflbm_lattice* L) {
  if (rflbm_status s = check_lattice(L)) return s;
  if (!L->have_plan) return RFLBM_OK;
  RFLBM_HIP(hipMemsetAsync(L->sk_sums, 0, 10 * L->nshells * sizeof(double), L->stream));
  RFLBM_HIP(hipMemsetAsync(L->sk_counts, 0, L->nshells * sizeof(unsigned long long), L->stream));
  L->sk_samples = 0;
  return RFLBM_OK;
}

rflbm_status rflbm_set_launch(rflbm_lattice* L, int32_t bx, int32_t xcd_remap) {
  if (rflbm_status s = check_lattice(L)) return s;
  if (bx != 64 && bx != 128 && bx != 256) return fail(RFLBM_EINVAL, "bx must be 64, 128 or 256");
  L->launch = make_launch(L->p.nx, L->p.ny, L->p.nz, bx, 256 / bx);
  L->xcd_remap = xcd_remap != 0;
  return RFLBM_OK;
}

rflbm_status rflbm_get_launch(const rflbm_lattice* L, int32_t* bx, int32_t* xcd_remap) {
  if (rflbm_status s = check_lattice(L)) return s;
  if (bx) *bx = static_cast<int32_t>(L->launch.bx);
  if (xcd_remap) *xcd_remap = L->xcd_remap ? 1 : 0;
  return RFLBM_OK;
}

rflbm_status rflbm_set_row_blocks(rflbm_lattice* L, int32_t enable) {
  if (rflbm_status s = check_lattice(L)) return s;
  L->row_mode = enable != 0;
  return RFLBM_OK;
}

rflbm_status rflbm_get_row_blocks(const rflbm_lattice* L, int32_t* active) {
  if (rflbm_status s = check_lattice(L)) return s;
  if (!active) return fail(RFLBM_EINVAL, "active is NULL");
  *active = odd_in_rows(L) ? 1 : 0;
  return RFLBM_OK;
}

rflbm_status rflbm_time_steps(rflbm_lattice* L, int64_t nsteps, double* ms) {
  if (rflbm_status s = check_lattice(L)) return s;
  if (L->is_view) return fail(RFLBM_ESTATE, "replicas of a batch are timed with rflbm_batch_time_steps");
  if (!ms) return fail(RFLBM_EINVAL, "ms is NULL");
  hipEvent_t e0, e1;
  RFLBM_HIP(hipEventCreate(&e0));
  if (const hipError_t c = hipEventCreate(&e1); c != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(RFLBM_EHIP, "hipEventCreate", c);
  }
  rflbm_status st = RFLBM_OK;
  hipError_t e = hipEventRecord(e0, L->stream);
  if (e == hipSuccess) {
    st = lattice_steps(L, nsteps);
    e = hipEventRecord(e1, L->stream);
  }
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float f = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(RFLBM_EHIP, "timing", e);
  if (st != RFLBM_OK) return st;
  *ms = f;
  return RFLBM_OK;
}

rflbm_status rflbm_rng_normals(uint64_t seed, uint32_t stream_id, uint32_t rounds, uint32_t node0,
                               uint32_t count, uint32_t t, float* u, float* z, void* hip_stream) {
  if (!u || !z) return fail(RFLBM_EINVAL, "u and z must be device arrays");
  if (rounds != 7 && rounds != 10) return fail(RFLBM_EINVAL, "rounds must be 7 or 10");
  RFLBM_HIP(launch_rng_normals(static_cast<uint32_t>(seed & 0xffffffffu), static_cast<uint32_t>(seed >> 32),
                               stream_id, static_cast<int>(rounds), node0, count, t, u, z,
                               static_cast<hipStream_t>(hip_stream)));
  return RFLBM_OK;
}

rflbm_status rflbm_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
  if (!dst || !src) return fail(RFLBM_EINVAL, "null pointer");
  if (bytes % 16 || reinterpret_cast<uintptr_t>(dst) % 16 || reinterpret_cast<uintptr_t>(src) % 16)
    return fail(RFLBM_EINVAL, "copy needs 16-byte aligned pointers and sizes");
  RFLBM_HIP(launch_copy(dst, src, bytes, static_cast<hipStream_t>(hip_stream)));
  return RFLBM_OK;
}

const char* rflbm_last_error(void) { return g_last_error.c_str(); }

const char* rflbm_version(void) { return "rflbm 0.1 (gfx950)"; }

}  // extern "C"
