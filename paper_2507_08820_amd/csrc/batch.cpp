// batch.cpp -- many independent Reg-FLBM boxes (replicas of different size, tau,
// k_BT and seed) stepped together by one persistent kernel launch per step,
// optionally replayed from a captured hipGraph of several steps, with a small
// autotuner for the launch shape.
//
// Each replica region of the batch buffer is laid out exactly like a
// stand-alone lattice (populations, flag, accumulators, partials), so a
// borrowed per-replica view supports every single-lattice call (readback,
// moments, S(k), set_populations).  After the replica regions come the batch
// tables: one ReplicaArgs per replica, the replica of each tile, the device
// step counter read by the kernel, and the per-tile statistics partials.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/rflbm.h"
#include "kernels.hpp"
#include "lattice.hpp"
#include "storage.hpp"

using namespace rflbm;

namespace {

constexpr uint32_t kTileChoices[2] = {128, 256};
constexpr int32_t kBpcChoices[5] = {0, 2, 4, 8, 16};

struct BatchLayout {
  std::vector<size_t> region_off;  // byte offset of each replica region
  size_t reps_off, tiles_off, step_off, partials_off, total;
  uint32_t max_tiles;              // tile-table capacity (smallest tile size)
};

BatchLayout batch_layout(int32_t n, const rflbm_params* p) {
  BatchLayout B;
  size_t off = 0;
  uint64_t tiles128 = 0;
  for (int32_t r = 0; r < n; ++r) {
    B.region_off.push_back(off);
    off += align_up(layout_for(p[r], false).total, kAlign);
    tiles128 += (node_count(p[r]) + 127) / 128;
  }
  B.max_tiles = static_cast<uint32_t>(tiles128);
  B.reps_off = off;
  off += align_up(static_cast<size_t>(n) * sizeof(ReplicaArgs), kAlign);
  B.tiles_off = off;
  off += align_up(static_cast<size_t>(B.max_tiles) * sizeof(uint32_t), kAlign);
  B.step_off = off;
  off += kAlign;
  B.partials_off = off;
  off += align_up(static_cast<size_t>(kNumStats) * B.max_tiles * sizeof(double), kAlign);
  B.total = off;
  return B;
}

std::string validate_batch(int32_t n, const rflbm_params* p) {
  if (n < 1 || n > 65535) return "replica count must be 1..65535";
  if (!p) return "params is NULL";
  uint64_t tiles = 0;
  for (int32_t r = 0; r < n; ++r) {
    const std::string e = validate(&p[r]);
    if (!e.empty()) return "replica " + std::to_string(r) + ": " + e;
    if (p[r].storage != p[0].storage) return "every replica must use the same storage type";
    if (p[r].philox_rounds != p[0].philox_rounds) return "every replica must use the same Philox rounds";
    if (static_cast<uint64_t>(p[r].nz) * plane_pitch_of(p[r]) >= (1ull << 32))
      return "replica " + std::to_string(r) + ": a batch replica must hold less than 4 GiB of populations";
    tiles += (node_count(p[r]) + 127) / 128;
  }
  if (tiles >= (1ull << 31)) return "too many nodes in the batch";
  return "";
}

}  // namespace

struct rflbm_batch {
  int32_t n = 0;
  std::vector<rflbm_params> p;
  BatchLayout B;
  uint8_t* buf = nullptr;
  bool owns_buf = false;
  hipStream_t stream = nullptr;
  std::vector<rflbm_lattice*> views;
  int64_t t = 0;
  uint32_t dev_step = 0;   // value of the device step counter once queued work has run
  int32_t stats_every = 0; // statistics every that many steps (0: off), all replicas
  int rounds = 0;          // Philox rounds of the kernel, 0 if every kT is 0
  uint32_t tile = 256;     // nodes per tile = threads per block
  int32_t bpc = 8;         // persistent blocks per CU (0: one block per tile)
  int32_t graph_steps = 0; // steps per captured graph (0: no graph)
  uint32_t ntiles = 0;
  bool all_ghost_eq = false;  // every replica has every omega_g = 1
  int cus = 0;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  int32_t exec_steps = 0;  // steps captured in exec
  int64_t exec_phase = 0;  // t mod stats_every at the first captured step
};

namespace {

rflbm_status check_batch(const rflbm_batch* b) {
  if (!b) return fail(RFLBM_EINVAL, "batch is NULL");
  return RFLBM_OK;
}

void drop_graph(rflbm_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->exec_steps = 0;
}

// (Re)writes the replica table and the tile table for the current tile size.
rflbm_status upload_tables(rflbm_batch* b) {
  std::vector<ReplicaArgs> reps(b->n);
  std::vector<uint32_t> tile_rep;
  uint32_t t0 = 0;
  bool all_geq = true;
  for (int32_t r = 0; r < b->n; ++r) {
    ReplicaArgs& ra = reps[r];
    std::memset(&ra, 0, sizeof(ra));
    ra.a = step_args(b->views[r]);
    all_geq = all_geq && ra.a.ghost_eq != 0u;
    const rflbm_params& p = b->p[r];
    ra.nodes = static_cast<uint32_t>(node_count(p));
    ra.tile0 = t0;
    ra.div_x = make_fastdiv(static_cast<uint32_t>(p.nx));
    ra.div_xy = make_fastdiv(static_cast<uint32_t>(p.nx) * static_cast<uint32_t>(p.ny));
    ra.acc = reinterpret_cast<double*>(b->views[r]->buf + b->views[r]->L.acc_off);
    const uint32_t nt = (ra.nodes + b->tile - 1) / b->tile;
    for (uint32_t k = 0; k < nt; ++k) tile_rep.push_back(static_cast<uint32_t>(r));
    t0 += nt;
  }
  b->ntiles = t0;
  b->all_ghost_eq = all_geq;
  RFLBM_HIP(hipMemcpyAsync(b->buf + b->B.reps_off, reps.data(), reps.size() * sizeof(ReplicaArgs),
                           hipMemcpyHostToDevice, b->stream));
  RFLBM_HIP(hipMemcpyAsync(b->buf + b->B.tiles_off, tile_rep.data(), tile_rep.size() * sizeof(uint32_t),
                           hipMemcpyHostToDevice, b->stream));
  RFLBM_HIP(hipStreamSynchronize(b->stream));
  drop_graph(b);
  return RFLBM_OK;
}

BatchArgs batch_args(const rflbm_batch* b, uint32_t step_offset) {
  BatchArgs a;
  a.reps = reinterpret_cast<const ReplicaArgs*>(b->buf + b->B.reps_off);
  a.tile_rep = reinterpret_cast<const uint32_t*>(b->buf + b->B.tiles_off);
  a.ntiles = b->ntiles;
  a.step = reinterpret_cast<const uint32_t*>(b->buf + b->B.step_off);
  a.step_offset = step_offset;
  a.partial_pitch = b->B.max_tiles;
  a.partials = reinterpret_cast<double*>(b->buf + b->B.partials_off);
  return a;
}

uint32_t* step_counter(rflbm_batch* b) { return reinterpret_cast<uint32_t*>(b->buf + b->B.step_off); }

bool stats_step(const rflbm_batch* b, int64_t t) { return b->stats_every > 0 && t % b->stats_every == 0; }

uint32_t batch_grid(const rflbm_batch* b) {
  if (b->bpc <= 0) return b->ntiles;
  const uint64_t g = static_cast<uint64_t>(b->bpc) * static_cast<uint64_t>(b->cus);
  return static_cast<uint32_t>(g < b->ntiles ? g : b->ntiles);
}

// Enqueues the step at time t, whose Philox step count is the device counter
// plus `offset`, with its statistics when t is a sampled step.
hipError_t enqueue_step(rflbm_batch* b, int64_t t, uint32_t offset, hipStream_t s) {
  const BatchArgs a = batch_args(b, offset);
  const bool stats = stats_step(b, t);
  hipError_t e = launch_batch_step(b->p[0].storage, (t & 1) != 0, b->rounds, b->all_ghost_eq, stats, a,
                                   batch_grid(b), b->tile, s);
  if (e == hipSuccess && stats) e = launch_batch_stats_reduce(a, static_cast<uint32_t>(b->n), b->tile, s);
  return e;
}

// Captures graph_steps steps starting at an even step count t0 into b->exec:
// step k reads the device counter plus k, and one last node advances the
// counter by graph_steps, so a replay needs the counter at t mod 2^32.  Which
// steps take statistics depends on t0 mod stats_every (kept in exec_phase).
rflbm_status build_graph(rflbm_batch* b, int64_t t0) {
  drop_graph(b);
  hipStream_t cap = nullptr;
  RFLBM_HIP(hipStreamCreate(&cap));
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  for (int32_t k = 0; e == hipSuccess && k < b->graph_steps; ++k)
    e = enqueue_step(b, t0 + k, static_cast<uint32_t>(k), cap);
  if (e == hipSuccess) e = launch_advance_step(step_counter(b), static_cast<uint32_t>(b->graph_steps), cap);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(cap, &g);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cap);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    b->exec = nullptr;
    return hip_fail(RFLBM_EHIP, "graph capture", e);
  }
  b->graph = g;
  b->exec_steps = b->graph_steps;
  b->exec_phase = b->stats_every > 0 ? t0 % b->stats_every : 0;
  return RFLBM_OK;
}

rflbm_status do_batch_steps(rflbm_batch* b, int64_t nsteps) {
  if (nsteps < 0) return fail(RFLBM_EINVAL, "nsteps must be >= 0");
  for (rflbm_lattice* v : b->views)
    if (v->t != b->t) return fail(RFLBM_ESTATE, "a replica was stepped or re-timed on its own");
  int64_t left = nsteps;
  rflbm_status st = RFLBM_OK;
  while (left > 0 && st == RFLBM_OK) {
    if (b->graph_steps > 0 && (b->t & 1) == 0 && left >= b->graph_steps) {
      const int64_t phase = b->stats_every > 0 ? b->t % b->stats_every : 0;
      if (b->exec_steps != b->graph_steps || b->exec_phase != phase) st = build_graph(b, b->t);
      if (st != RFLBM_OK) break;
      const uint32_t t32 = static_cast<uint32_t>(b->t & 0xffffffffu);
      if (b->dev_step != t32) {
        if (const hipError_t e = launch_set_u32(step_counter(b), t32, b->stream); e != hipSuccess) {
          st = hip_fail(RFLBM_EHIP, "step counter", e);
          break;
        }
        b->dev_step = t32;
      }
      if (const hipError_t e = hipGraphLaunch(b->exec, b->stream); e != hipSuccess) {
        st = hip_fail(RFLBM_EHIP, "hipGraphLaunch", e);
        break;
      }
      b->dev_step += static_cast<uint32_t>(b->graph_steps);
      b->t += b->graph_steps;
      left -= b->graph_steps;
    } else {
      // outside a graph the step count goes in as the offset from the counter
      const uint32_t offset = static_cast<uint32_t>(b->t & 0xffffffffu) - b->dev_step;
      if (const hipError_t e = enqueue_step(b, b->t, offset, b->stream); e != hipSuccess) {
        st = hip_fail(RFLBM_EHIP, "batch step", e);
        break;
      }
      b->t += 1;
      left -= 1;
    }
  }
  // the replicas share the batch's step count, also after a failed launch
  for (rflbm_lattice* v : b->views) v->t = b->t;
  return st;
}

rflbm_status time_batch(rflbm_batch* b, int64_t nsteps, double* ms) {
  hipEvent_t e0, e1;
  RFLBM_HIP(hipEventCreate(&e0));
  if (const hipError_t c = hipEventCreate(&e1); c != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(RFLBM_EHIP, "hipEventCreate", c);
  }
  hipError_t e = hipEventRecord(e0, b->stream);
  rflbm_status st = RFLBM_OK;
  if (e == hipSuccess) {
    st = do_batch_steps(b, nsteps);
    e = hipEventRecord(e1, b->stream);
  }
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float f = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != RFLBM_OK) return st;
  if (e != hipSuccess) return hip_fail(RFLBM_EHIP, "timing", e);
  *ms = f;
  return RFLBM_OK;
}

std::string batch_signature(const rflbm_batch* b) {
  // FNV-1a over the replica boxes; storage and count spelled out
  uint64_t h = 1469598103934665603ull;
  for (const rflbm_params& p : b->p)
    for (int32_t d : {p.nx, p.ny, p.nz}) {
      h ^= static_cast<uint64_t>(d);
      h *= 1099511628211ull;
    }
  char s[96];
  std::snprintf(s, sizeof(s), "gfx950:s%d:r%d:n%d:%016llx", b->p[0].storage, b->rounds, b->n,
                static_cast<unsigned long long>(h));
  return s;
}

}  // namespace

extern "C" {

size_t rflbm_batch_required_bytes(int32_t n, const rflbm_params* p) {
  if (!validate_batch(n, p).empty()) return 0;
  return batch_layout(n, p).total;
}

rflbm_status rflbm_batch_create(int32_t n, const rflbm_params* p, void* dev_buf, size_t bytes, void* hip_stream,
                                rflbm_batch** out) {
  if (!out) return fail(RFLBM_EINVAL, "out is NULL");
  *out = nullptr;
  const std::string err = validate_batch(n, p);
  if (!err.empty()) return fail(RFLBM_EINVAL, err);
  const BatchLayout B = batch_layout(n, p);
  if (dev_buf && bytes < B.total) return fail(RFLBM_ENOMEM, "caller buffer smaller than rflbm_batch_required_bytes");
  if (dev_buf && (reinterpret_cast<uintptr_t>(dev_buf) % kAlign) != 0)
    return fail(RFLBM_EINVAL, "caller buffer must be 256-byte aligned");
  rflbm_batch* b = new (std::nothrow) rflbm_batch();
  if (!b) return fail(RFLBM_ENOMEM, "host allocation failed");
  b->n = n;
  b->p.assign(p, p + n);
  b->B = B;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->rounds = 0;
  for (const rflbm_params& q : b->p)
    if (q.kT > 0.0) b->rounds = static_cast<int>(q.philox_rounds);
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || b->cus <= 0)
    b->cus = 256;
  if (dev_buf) {
    b->buf = static_cast<uint8_t*>(dev_buf);
  } else {
    void* m = nullptr;
    const hipError_t e = hipMalloc(&m, B.total);
    if (e != hipSuccess) {
      delete b;
      return hip_fail(RFLBM_ENOMEM, "hipMalloc", e);
    }
    b->buf = static_cast<uint8_t*>(m);
    b->owns_buf = true;
  }
  for (int32_t r = 0; r < n; ++r) {
    rflbm_lattice* v = new (std::nothrow) rflbm_lattice();
    if (!v) {
      rflbm_batch_destroy(b);
      return fail(RFLBM_ENOMEM, "host allocation failed");
    }
    lattice_init(v, p[r], b->buf + B.region_off[r], b->stream, false);  // plain layout
    v->is_view = true;
    b->views.push_back(v);
    if (lattice_clear(v) != hipSuccess) {
      rflbm_batch_destroy(b);
      return fail(RFLBM_EHIP, "clearing a replica failed");
    }
  }
  if (launch_fill_zero(reinterpret_cast<double*>(b->buf + B.step_off), 1, b->stream) != hipSuccess) {
    rflbm_batch_destroy(b);
    return fail(RFLBM_EHIP, "clearing the step counter failed");
  }
  if (rflbm_status s = upload_tables(b)) {
    rflbm_batch_destroy(b);
    return s;
  }
  *out = b;
  return RFLBM_OK;
}

rflbm_status rflbm_batch_destroy(rflbm_batch* b) {
  if (!b) return RFLBM_OK;
  (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  for (rflbm_lattice* v : b->views) {
    lattice_release(v);
    delete v;
  }
  if (b->owns_buf) (void)hipFree(b->buf);
  delete b;
  return RFLBM_OK;
}

rflbm_status rflbm_batch_lattice(rflbm_batch* b, int32_t r, rflbm_lattice** view) {
  if (rflbm_status s = check_batch(b)) return s;
  if (!view || r < 0 || r >= b->n) return fail(RFLBM_EINVAL, "replica index out of range");
  *view = b->views[r];
  return RFLBM_OK;
}

rflbm_status rflbm_batch_set_params(rflbm_batch* b, int32_t r, const rflbm_params* p) {
  if (rflbm_status s = check_batch(b)) return s;
  if (r < 0 || r >= b->n) return fail(RFLBM_EINVAL, "replica index out of range");
  if (!p) return fail(RFLBM_EINVAL, "params is NULL");
  if (p->philox_rounds != b->p[0].philox_rounds)
    return fail(RFLBM_EINVAL, "every replica must use the same Philox rounds");
  if (rflbm_status s = lattice_set_params(b->views[r], p)) return s;
  b->p[r] = *p;
  int rounds = 0;
  for (const rflbm_params& q : b->p)
    if (q.kT > 0.0) rounds = static_cast<int>(q.philox_rounds);
  b->rounds = rounds;
  return upload_tables(b);
}

rflbm_status rflbm_batch_step(rflbm_batch* b, int64_t nsteps) {
  if (rflbm_status s = check_batch(b)) return s;
  return do_batch_steps(b, nsteps);
}

rflbm_status rflbm_batch_step_separate(rflbm_batch* b, int64_t nsteps) {
  if (rflbm_status s = check_batch(b)) return s;
  if (nsteps < 0) return fail(RFLBM_EINVAL, "nsteps must be >= 0");
  for (rflbm_lattice* v : b->views)
    if (v->t != b->t) return fail(RFLBM_ESTATE, "a replica was stepped or re-timed on its own");
  for (int64_t k = 0; k < nsteps; ++k) {
    for (rflbm_lattice* v : b->views)
      if (rflbm_status s = lattice_steps(v, 1)) return s;
    b->t += 1;
  }
  return RFLBM_OK;
}

rflbm_status rflbm_batch_set_step_count(rflbm_batch* b, int64_t t) {
  if (rflbm_status s = check_batch(b)) return s;
  if (t < 0) return fail(RFLBM_EINVAL, "step count must be >= 0");
  // one scratch plane for the largest replica, taken before any replica moves,
  // so that running out of memory leaves the whole batch unchanged
  void* tmp = nullptr;
  if ((t & 1) != (b->t & 1)) {
    size_t bytes = 0;
    for (rflbm_lattice* v : b->views) bytes = std::max(bytes, parity_scratch_bytes(v));
    if (const hipError_t m = hipMalloc(&tmp, bytes); m != hipSuccess)
      return hip_fail(RFLBM_ENOMEM, "re-layout scratch", m);
  }
  rflbm_status st = RFLBM_OK;
  for (rflbm_lattice* v : b->views)
    if ((st = lattice_set_step_count_with(v, t, tmp)) != RFLBM_OK) break;
  if (tmp) (void)hipFree(tmp);
  if (st != RFLBM_OK) return st;
  b->t = t;
  return RFLBM_OK;
}

rflbm_status rflbm_batch_stats_config(rflbm_batch* b, int32_t every) {
  if (rflbm_status s = check_batch(b)) return s;
  if (every < 0) return fail(RFLBM_EINVAL, "every must be >= 0");
  b->stats_every = every;
  // rflbm_batch_step_separate steps the views as single lattices
  for (rflbm_lattice* v : b->views) v->stats_every = every;
  drop_graph(b);
  return RFLBM_OK;
}

rflbm_status rflbm_batch_sync(rflbm_batch* b) {
  if (rflbm_status s = check_batch(b)) return s;
  RFLBM_HIP(hipStreamSynchronize(b->stream));
  for (int32_t r = 0; r < b->n; ++r) {
    const rflbm_status s = rflbm_sync(b->views[r]);
    if (s == RFLBM_EUNSTABLE) return fail(RFLBM_EUNSTABLE, "replica " + std::to_string(r) + " became unstable");
    if (s != RFLBM_OK) return s;
  }
  return RFLBM_OK;
}

int64_t rflbm_batch_step_count(const rflbm_batch* b) { return b ? b->t : -1; }

int64_t rflbm_batch_nodes(const rflbm_batch* b) {
  if (!b) return -1;
  int64_t s = 0;
  for (const rflbm_params& p : b->p) s += static_cast<int64_t>(node_count(p));
  return s;
}

rflbm_status rflbm_batch_set_launch(rflbm_batch* b, int32_t tile, int32_t blocks_per_cu, int32_t graph_steps) {
  if (rflbm_status s = check_batch(b)) return s;
  if (tile != 128 && tile != 256) return fail(RFLBM_EINVAL, "tile must be 128 or 256 nodes");
  if (blocks_per_cu < 0 || blocks_per_cu > 64) return fail(RFLBM_EINVAL, "blocks_per_cu must be 0..64");
  if (graph_steps < 0 || (graph_steps % 2) != 0 || graph_steps > 4096)
    return fail(RFLBM_EINVAL, "graph_steps must be an even number 0..4096");
  const bool retile = static_cast<uint32_t>(tile) != b->tile;
  b->tile = static_cast<uint32_t>(tile);
  b->bpc = blocks_per_cu;
  b->graph_steps = graph_steps;
  drop_graph(b);
  if (retile) return upload_tables(b);
  return RFLBM_OK;
}

rflbm_status rflbm_batch_get_launch(const rflbm_batch* b, int32_t* tile, int32_t* blocks_per_cu,
                                    int32_t* graph_steps) {
  if (rflbm_status s = check_batch(b)) return s;
  if (tile) *tile = static_cast<int32_t>(b->tile);
  if (blocks_per_cu) *blocks_per_cu = b->bpc;
  if (graph_steps) *graph_steps = b->graph_steps;
  return RFLBM_OK;
}

rflbm_status rflbm_batch_time_steps(rflbm_batch* b, int64_t nsteps, double* ms) {
  if (rflbm_status s = check_batch(b)) return s;
  if (!ms) return fail(RFLBM_EINVAL, "ms is NULL");
  return time_batch(b, nsteps, ms);
}

rflbm_status rflbm_batch_autotune(rflbm_batch* b, int32_t trial_steps, const char* cache_path) {
  if (rflbm_status s = check_batch(b)) return s;
  if (trial_steps < 2 || (trial_steps % 2) != 0) return fail(RFLBM_EINVAL, "trial_steps must be even and >= 2");
  const std::string sig = batch_signature(b);
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string key;
      int32_t tile = 0, bpc = -1;
      if ((ls >> key >> tile >> bpc) && key == sig)
        return rflbm_batch_set_launch(b, tile, bpc, b->graph_steps);
    }
  }
  // the trials step a saved copy's original: every replica region (populations,
  // flags, accumulators) is copied aside first and put back afterwards, with
  // the step count, so a tuned batch continues exactly as an untuned one
  const size_t state_bytes = b->B.reps_off;
  void* saved = nullptr;
  if (const hipError_t m = hipMalloc(&saved, state_bytes); m != hipSuccess)
    return hip_fail(RFLBM_ENOMEM, "autotune state copy", m);
  hipError_t ce = hipMemcpyAsync(saved, b->buf, state_bytes, hipMemcpyDeviceToDevice, b->stream);
  if (ce == hipSuccess) ce = hipStreamSynchronize(b->stream);
  if (ce != hipSuccess) {
    (void)hipFree(saved);
    return hip_fail(RFLBM_EHIP, "autotune state copy", ce);
  }
  const int64_t t0 = b->t;
  const int32_t keep_graph = b->graph_steps, keep_tile = static_cast<int32_t>(b->tile), keep_bpc = b->bpc;
  const int32_t keep_stats = b->stats_every;
  (void)rflbm_batch_stats_config(b, 0);  // trials time plain steps
  double best = 1e300;
  int32_t best_tile = keep_tile, best_bpc = keep_bpc;
  rflbm_status st = RFLBM_OK;
  for (uint32_t tile : kTileChoices) {
    for (int32_t bpc : kBpcChoices) {
      if ((st = rflbm_batch_set_launch(b, static_cast<int32_t>(tile), bpc, 0)) != RFLBM_OK) break;
      double ms = 0.0;
      if ((st = time_batch(b, 2, &ms)) != RFLBM_OK) break;  // warm-up
      if ((st = time_batch(b, trial_steps, &ms)) != RFLBM_OK) break;
      if (ms < best) {
        best = ms;
        best_tile = static_cast<int32_t>(tile);
        best_bpc = bpc;
      }
    }
    if (st != RFLBM_OK) break;
  }
  // restore the state and step count (every trial ran an even number of steps,
  // so the stored layout has the parity of t0)
  ce = hipMemcpyAsync(b->buf, saved, state_bytes, hipMemcpyDeviceToDevice, b->stream);
  if (ce == hipSuccess) ce = hipStreamSynchronize(b->stream);
  (void)hipFree(saved);
  b->t = t0;
  for (rflbm_lattice* v : b->views) v->t = t0;
  (void)rflbm_batch_stats_config(b, keep_stats);
  if (ce != hipSuccess) return hip_fail(RFLBM_EHIP, "autotune state restore", ce);
  if (st != RFLBM_OK) {
    (void)rflbm_batch_set_launch(b, keep_tile, keep_bpc, keep_graph);
    return st;
  }
  if (rflbm_status s = rflbm_batch_set_launch(b, best_tile, best_bpc, keep_graph)) return s;
  if (cache_path) {
    std::ofstream outf(cache_path, std::ios::app);
    if (outf) outf << sig << ' ' << best_tile << ' ' << best_bpc << ' ' << best / trial_steps << '\n';
  }
  return RFLBM_OK;
}

}  // extern "C"
