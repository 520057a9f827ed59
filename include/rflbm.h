/*
 * rflbm.h -- C interface of librflbm, a single-GPU (MI355X, gfx950) library for
 * the regularized fluctuating lattice Boltzmann method (Reg-FLBM) on the D3Q27
 * lattice of Lauricella, Montessori, Tiribocchi and Succi, "Regularized
 * Fluctuating Lattice Boltzmann Model" (arXiv:2507.08820).
 *
 * The model (Sec. II).  Each node of a periodic nx x ny x nz box carries the 27
 * populations f_i of Table I.  One step t -> t + 1 projects f onto the 27
 * Hermite modes of Table II (Eq. moments), rebuilds the equilibrium modes from
 * rho and u (Eq. rec-eq), relaxes the second-order non-equilibrium modes
 * (k = 4..9) with omega_h and the ghost modes (k = 10..26) with omega_g, adds
 * Gaussian noise phi_k r_k to every non-conserved mode with the amplitude of
 * Eq. fluct_phi, transforms back (Eq. backtrasf) and streams
 * f_i(x + c_i, t + 1) = f*_i(x, t) (Eqs. eq:streaming, r-flbe2).  With
 * omega_g = 1 and equal bulk and shear rates this is exactly Eq. r-flbe2.  The
 * BGK-FLBM comparator of Eq. flbe (Sec. III) is the same update with every
 * non-conserved mode relaxed by one omega.
 *
 * Conventions shared by every call.
 *   Population order: i = (c_x + 1) + 3 (c_y + 1) + 9 (c_z + 1), so the
 *     opposite of i is 26 - i and i = 13 is the rest population.
 *   Node order: n = x + nx (y + ny z); N = nx ny nz must be below 2^32 and
 *     one z plane of populations (27 nx ny values) below 4 GiB.
 *   Population arrays exchanged with the caller are FP64, planar:
 *     f[i * N + n], i = 0..26, and hold the pre-collision state f(x, t) at the
 *     current step count t.
 *   Random numbers (r_k ~ N(0, 1) of Eq. fluct_phi; the paper leaves the
 *     generator open): Philox4x32 with key (seed low word, seed high word) and
 *     counter (n, t mod 2^32, j = 0..3, stream_id); the words w0..w3 of call
 *     j carry Box-Muller pairs 3 j + m, m = 0..2: radius uniform 1 - b 2^-23
 *     from the top 23 bits b = w_m >> 9, angle uniform a 2^-16 from
 *     a = w3 >> 16, w3 & 0xFFFF and (w0 & 0xFF) 2^8 + (w1 & 0xFF) for
 *     m = 0, 1, 2; pair p gives normals z_2p, z_2p+1, and mode k (Table II
 *     order, 4..26) receives z_(k-4).  The trajectory is therefore a function of (params, initial
 *     state) only, on any device or host.
 *   Memory: "device" pointers are HIP device allocations (for instance torch
 *     tensors on the GPU); "host" pointers are ordinary memory.  Host arrays
 *     are read or written synchronously before the call returns.  Device
 *     arrays are read or written in stream order on the lattice's stream.
 *   Streams: every lattice works on the HIP stream given at creation (NULL:
 *     the null stream).  All calls except rflbm_sync, readbacks into host
 *     memory and rflbm_time_steps return without waiting for the GPU.
 *   Errors: every call returns an rflbm_status; no C++ exception crosses this
 *     interface.  A failed call leaves the lattice unchanged unless stated.
 *     rflbm_last_error() gives a text for the last failure on the calling
 *     thread.
 */
#ifndef RFLBM_H
#define RFLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rflbm_lattice rflbm_lattice;

typedef enum {
  RFLBM_OK = 0,
  RFLBM_EINVAL = -1,    /* bad argument (sizes, tau <= 1/2, null pointer, ...) */
  RFLBM_ENOMEM = -2,    /* device allocation failed or caller buffer too small */
  RFLBM_EHIP = -3,      /* a HIP runtime call failed (text in rflbm_last_error) */
  RFLBM_EUNSTABLE = -4, /* a node reached rho <= 0 or a non-finite value */
  RFLBM_ESTATE = -5     /* call not valid in the lattice's current state */
} rflbm_status;

/* Storage of the populations in device memory.  All three store the deviation
 * f_i - w_i rho0; F16 and BF16 store it in units of
 * sigma_i = sqrt(w_i) * scale, scale = sqrt(rho0 kT / cs^2) (the thermal
 * standard deviation, Eq. fluct_phi with the stationary covariance
 * rho0 kT w_i / cs^2), or storage_scale when that is set.  Collision arithmetic
 * is FP32 for every storage type; stores round to nearest even. */
typedef enum { RFLBM_F32 = 0, RFLBM_F16 = 1, RFLBM_BF16 = 2 } rflbm_storage;

typedef enum {
  RFLBM_MODEL_REG = 0, /* Reg-FLBM, Eq. r-flbe2; ghosts k = 10..26 relax their
                          projected non-equilibrium m_k - m_eq,k by (1 - omega_g,k) */
  RFLBM_MODEL_BGK = 1, /* BGK-FLBM, Eq. flbe (full-Hermite equilibrium, one tau) */
  RFLBM_MODEL_REC = 2  /* Reg-FLBM whose ghost non-equilibrium is rebuilt from the
                          second-order one and u by the recursion of
                          Eq. recursive_eq (Sec. II.B), then relaxed by
                          (1 - omega_g,k) with the noise of Eq. fluct_phi; read
                          as the sum over index pairs
                          a1_(s1..sn) = sum_{i<j} a1_(si sj) prod_{l != i,j} u_sl.
                          Equal to RFLBM_MODEL_REG when every omega_g = 1; for
                          omega_g != 1 it does not balance the ghost noise
                          (linearised variance deficit mu b_k (1 - omega_g)^2 per
                          ghost mode) */
} rflbm_model;

typedef struct {
  int32_t nx, ny, nz;      /* periodic box, each >= 2 (fixed at creation) */
  int32_t storage;         /* rflbm_storage (fixed at creation) */
  int32_t model;           /* rflbm_model */
  uint32_t philox_rounds;  /* Philox rounds, 7 or 10 (else EINVAL); 7 is the default */
  double rho0;             /* reference density > 0 (Sec. III: rho normalised to 1) */
  double kT;               /* k_B T >= 0; 0 gives the deterministic Reg-LBM (Sec. IV) */
  double tau_shear;        /* 1/omega_h on the deviatoric modes k = 4..9, > 1/2; the
                              BGK model uses it for every mode */
  double tau_bulk;         /* 1/omega on the trace of the xx, yy, zz block, > 1/2 */
  double tau_ghost[17];    /* 1/omega_g for k = 10..26, > 1/2 (paper: 1, Sec. II.B) */
  uint64_t seed;           /* Philox key */
  uint32_t stream_id;      /* fourth Philox counter word (replica id), 0 by default */
  uint32_t reserved;       /* must be 0 */
  double storage_scale;    /* F16/BF16 deviation unit; 0 selects the thermal scale,
                              which needs kT > 0 */
} rflbm_params;

/* Fills p with defaults for an nx x ny x nz box: F32, Reg model, 7 Philox
 * rounds, rho0 = 1, kT = 0, every tau = 1, seed 1, stream 0. */
void rflbm_params_default(rflbm_params* p, int32_t nx, int32_t ny, int32_t nz);

/* Bytes of device memory a lattice with these parameters needs (populations,
 * statistics partials, flags), or 0 if the parameters are invalid. */
size_t rflbm_required_bytes(const rflbm_params* p);

/* Creates a lattice: the periodic box and the parameters of the update of
 * Sec. II (tau_h, omega_g, k_BT of Eq. fluct_phi) and of the validation runs
 * of Sec. III (cubic periodic box, rho normalised to rho0).  dev_buf: device memory of at least
 * rflbm_required_bytes(p) bytes that the caller owns and keeps alive until
 * rflbm_destroy (the library never frees it), or NULL to let the library
 * allocate it.  hip_stream: a hipStream_t or NULL.  The populations start at
 * rest equilibrium f_i = w_i rho0, step count 0.  Returns EINVAL for invalid
 * parameters, ENOMEM if bytes is too small or allocation fails. */
rflbm_status rflbm_create(const rflbm_params* p, void* dev_buf, size_t bytes, void* hip_stream,
                          rflbm_lattice** out);

/* Waits for the lattice's stream, then releases the lattice (and its buffer if
 * the library allocated it).  NULL is accepted. */
rflbm_status rflbm_destroy(rflbm_lattice* lat);

/* Replaces the physical parameters of the update of Sec. II (model, tau_h
 * and omega_g of Eq. r-flbe2, k_BT of Eq. fluct_phi, rho0 of Sec. III) and of
 * the noise source (rounds, seed, stream id), and the storage scale.  Box size and storage type must not change
 * (EINVAL).  Changing rho0 or the 16-bit storage scale re-encodes the stored
 * populations so that the state f is kept. */
rflbm_status rflbm_set_params(rflbm_lattice* lat, const rflbm_params* p);
rflbm_status rflbm_get_params(const rflbm_lattice* lat, rflbm_params* p);

/* Sets f to the full-Hermite equilibrium f^(0)(rho, u) of Eq. hermite_feq2 at
 * every node.  rho: N values or NULL (rho0 everywhere); u: 3N values, planar
 * (u[a * N + n]), or NULL (zero).  FP64, host memory if host_ptrs != 0, else
 * device memory.  The step count is kept. */
rflbm_status rflbm_init_equilibrium(rflbm_lattice* lat, const double* rho, const double* u,
                                    int host_ptrs);

/* Thermalised start: f_i = f^(0)_i(rho, u) + sqrt(rho0 kT w_i / cs^2) xi_i,
 * the stationary covariance of the fluctuating update in the linear regime
 * (Eq. fluct_phi), so that statistics need no equilibration transient.  xi_i
 * is normal i of the node's Philox/Box-Muller stream at the reserved step word
 * 0xFFFFFFFF (calls j = 0..4; 27 of 30 normals used), keyed like the step's
 * noise.  Arguments as for rflbm_init_equilibrium. */
rflbm_status rflbm_init_thermal(rflbm_lattice* lat, const double* rho, const double* u,
                                int host_ptrs);

/* Advances nsteps >= 0 time steps (one fused stream-and-collide kernel per
 * step, Eq. r-flbe2).  Asynchronous on the lattice stream.  Instability is
 * reported by the next rflbm_sync. */
rflbm_status rflbm_step(rflbm_lattice* lat, int64_t nsteps);

/* Build addition (no passage of the paper defines it): waits for the lattice
 * stream.  Returns EUNSTABLE if any node of any step so
 * far saw rho <= 0 or a non-finite density or momentum (the flag is sticky
 * until the populations are set again). */
rflbm_status rflbm_sync(rflbm_lattice* lat);

/* Steps taken so far: the time t of the state f(x, t) of Eq. eq:streaming,
 * which is also the step word of the noise counter. */
int64_t rflbm_step_count(const rflbm_lattice* lat);
/* Sets the time t of Eq. eq:streaming (checkpoint restart: set_populations + set_step_count resumes a run
 * bit for bit, since the noise depends only on (seed, n, t, stream_id)).  A
 * change of parity moves the stored state to the other AA layout in place and
 * bit for bit, with a temporary device buffer of one population plane
 * (nx ny nz stored words), freed before the call returns.  ENOMEM (no room for
 * that buffer) leaves the lattice unchanged; after an EHIP during the move the
 * stored populations are undefined until they are set again. */
rflbm_status rflbm_set_step_count(rflbm_lattice* lat, int64_t t);

/* Reads the pre-collision populations f_i(x, t) of Eq. eq:streaming (the
 * state after t complete steps; Table I velocity order as above; FP64, planar,
 * 27 N values) into dst.  With a host dst the call waits for the stream. */
rflbm_status rflbm_get_populations(rflbm_lattice* lat, double* dst, int dst_is_host);
/* Reads f(x, t) at `count` nodes only: nodes[k] (device array of node indices
 * n < N) -> dst[i * count + k] (device, FP64, 27 * count values).  For
 * checking large boxes against a reference one node at a time.  An index
 * n >= N reads nothing and yields NaN for its 27 values. */
rflbm_status rflbm_get_populations_at(rflbm_lattice* lat, const uint32_t* nodes, uint32_t count,
                                      double* dst);
/* Writes the pre-collision populations f_i(x, t) of Eq. eq:streaming from src
 * (FP64, planar, 27 N values); clears the instability flag. */
rflbm_status rflbm_set_populations(rflbm_lattice* lat, const double* src, int src_is_host);

/* Moment fields of the current state, FP32, planar.  mask selects fields in
 * this order: RFLBM_M_RHO (rho), RFLBM_M_J (rho u_x, rho u_y, rho u_z),
 * RFLBM_M_PI (Pi_xx, Pi_yy, Pi_zz, Pi_xy, Pi_xz, Pi_yz) with
 * Pi_ab = sum_i f_i H^(2)_i,ab = a0^(2) + a1^(2), the momentum flux of Sec. III;
 * dst holds (number of selected fields) * N floats. */
#define RFLBM_M_RHO 1u
#define RFLBM_M_J 2u
#define RFLBM_M_PI 4u
rflbm_status rflbm_get_moments(rflbm_lattice* lat, uint32_t mask, float* dst, int dst_is_host);

/* For callers that cannot allocate device memory (serving loops, harnesses
 * that forbid hipMalloc, code around HIP graph captures): the fields of
 * rflbm_get_moments (same mask, same planar layout, bit for bit the same
 * values) into HOST memory dst, which the caller owns and sizes to
 * (number of selected fields) * N floats.  rflbm_get_moments with a host dst
 * stages the fields in a device buffer of the whole field size that it
 * allocates per call; this call allocates nothing: the fields pass through a
 * fixed 8 MiB device array that the library holds on each GPU it runs on until
 * the process ends, in chunks of at most 8 MiB, so every box size is served.
 * Runs on the lattice's stream and waits for it before returning.  Calls on
 * one GPU share that array and are serialised by the library (one at a time
 * per GPU in a process).  EINVAL for a NULL lattice or dst or a bad mask; EHIP
 * if a kernel or copy fails (dst then partly written). */
rflbm_status rflbm_get_moments_host_noalloc(rflbm_lattice* lat, uint32_t mask, float* dst);

/* Ensemble statistics of Sec. III (equilibration ratios), accumulated on the
 * GPU in FP64 inside the step kernel on every step whose count t is a multiple
 * of `every` (sampled before that step's collision).  Sums run over sampled
 * steps and all nodes:  drho = rho - rho0, j = rho u, u2 = u_a^2 with
 * u = j / rho, pi = Pi_ab in the order xx, yy, zz, xy, xz, yz.  The reduction
 * order is fixed, so results are reproducible bit for bit.  mass_dev and
 * momentum are sum_n drho and sum_n j at the last sampled step. */
typedef struct {
  int64_t samples;
  int64_t nodes;
  double sum_drho, sum_drho2;
  double sum_j[3], sum_j2[3];
  double sum_u2[3];
  double sum_pi[6], sum_pi2[6];
  double mass_dev;
  double momentum[3];
} rflbm_stats;

/* every = 0 disables sampling. */
rflbm_status rflbm_stats_config(rflbm_lattice* lat, int32_t every);
/* Waits for the stream and copies the accumulators. */
rflbm_status rflbm_get_stats(rflbm_lattice* lat, rflbm_stats* out);
rflbm_status rflbm_reset_stats(rflbm_lattice* lat);

/* Static structure factor (Sec. III, normalised FFT): for each of the 10 moment
 * fields of rflbm_get_moments (rho, j_x, j_y, j_z, Pi_xx, ..., Pi_yz), the
 * current field's fluctuation dm is Fourier transformed with
 * dm^(n) = N^-1/2 sum_x dm(x) exp(-2 pi i n.x / L) and |dm^(n)|^2 is added
 * to the FP64 sum of shell round(|n|), n_a in (-L_a/2, L_a/2], n = 0 left
 * out (for non-cubic boxes the shell uses the integer vector n).  Device
 * scratch for the transforms is allocated by the library on first use and
 * kept until rflbm_destroy. */
rflbm_status rflbm_sk_sample(rflbm_lattice* lat);
/* Number of shells (round(|n|) of the largest |n|, plus one). */
int32_t rflbm_sk_nshells(const rflbm_lattice* lat);
/* Copies the shell sums of one field (0..9) and the number of wavevectors per
 * shell (per sample) into host arrays of nshells entries; *samples gets the
 * number of rflbm_sk_sample calls since the last reset. */
rflbm_status rflbm_get_sk(rflbm_lattice* lat, int32_t field, double* shell_sum,
                          int64_t* shell_count, int32_t nshells, int64_t* samples);
rflbm_status rflbm_reset_sk(rflbm_lattice* lat);

/* Launch shape of the step kernel: blocks of bx x (256 / bx) nodes of one
 * z plane, bx in {64, 128, 256}; xcd_remap != 0 hands each of the 8 XCDs a
 * contiguous range of tiles (neighbouring tiles then share an L2).  Any shape
 * gives the same results bit for bit.  rflbm_create picks the widest bx that
 * the box's x extent fills. */
rflbm_status rflbm_set_launch(rflbm_lattice* lat, int32_t bx, int32_t xcd_remap);
rflbm_status rflbm_get_launch(const rflbm_lattice* lat, int32_t* bx, int32_t* xcd_remap);

/* Row-aligned blocks for the steps without statistics (the streaming of
 * Eq. eq:streaming in its two AA phases), used where the step is bound by
 * bandwidth: FP32 storage, or k_BT = 0.  When enabled and nx is a multiple of
 * 64, every even step runs one 64-node x-segment per block, and every odd step
 * one block per x-row (if nx <= 1024).  The shifts by c_x = +-1 then stay
 * inside a block (values move between lanes), and every load and store covers
 * whole aligned cache lines.  The 16-bit steps with noise are bound by
 * arithmetic and keep the tiled kernel.  Statistics steps, and all steps when
 * disabled, keep the tiled shape of rflbm_set_launch.  Results are bit for bit
 * the same either way.  Enabled by rflbm_create.  rflbm_get_row_blocks sets
 * *active to 1 when the next odd step runs in whole rows (it depends on
 * storage, k_BT and nx). */
rflbm_status rflbm_set_row_blocks(rflbm_lattice* lat, int32_t enable);
rflbm_status rflbm_get_row_blocks(const rflbm_lattice* lat, int32_t* active);

/* Times nsteps steps with HIP events recorded on the lattice's own stream and
 * waits for them; *ms gets the elapsed milliseconds.  Used by benchmarks. */
rflbm_status rflbm_time_steps(rflbm_lattice* lat, int64_t nsteps, double* ms);

/* ------------------------------------------------------------------------
 * Batched replicas.  Fluctuation statistics need many independent noise
 * realisations; a batch holds n boxes (each with its own size, taus, k_BT,
 * rho0, seed and stream id, one common storage type and Philox round count) in
 * one buffer and advances all of them by one persistent kernel launch per step
 * (Eq. r-flbe2 at every node of every replica).  Replica r evolves exactly as a
 * stand-alone lattice with params p[r] would, bit for bit.
 * Every replica shares the batch's step count t; each replica must hold less
 * than 4 GiB of populations. */
typedef struct rflbm_batch rflbm_batch;

/* Device bytes for n replicas with params p[0..n-1], 0 if invalid. */
size_t rflbm_batch_required_bytes(int32_t n, const rflbm_params* p);
/* Creates a batch (buffer ownership and stream as for rflbm_create); every
 * replica starts at rest, t = 0.  EINVAL if any params are invalid or if the
 * replicas differ in storage type or Philox rounds. */
rflbm_status rflbm_batch_create(int32_t n, const rflbm_params* p, void* dev_buf, size_t bytes,
                                void* hip_stream, rflbm_batch** out);
/* Waits for the stream and releases the batch and its replica views. */
rflbm_status rflbm_batch_destroy(rflbm_batch* b);
/* Borrowed view of replica r: every rflbm_* lattice call that reads or writes
 * state works on it (populations, moments, S(k), init, set_populations,
 * statistics readback and reset); stepping, re-timing, parameter changes and
 * the statistics schedule go through the batch (the lattice calls return
 * ESTATE on a view).  The view lives as long as the batch; rflbm_destroy on it
 * returns ESTATE. */
rflbm_status rflbm_batch_lattice(rflbm_batch* b, int32_t r, rflbm_lattice** view);
/* Replaces the parameters of replica r (same rules as rflbm_set_params). */
rflbm_status rflbm_batch_set_params(rflbm_batch* b, int32_t r, const rflbm_params* p);
/* Advances every replica nsteps steps: one persistent launch per step, or
 * replays of a captured graph of graph_steps steps (rflbm_batch_set_launch)
 * whenever t is even.  Asynchronous on the batch stream. */
rflbm_status rflbm_batch_step(rflbm_batch* b, int64_t nsteps);
/* The same update with one single-box launch per replica and step (the
 * reference the persistent form is measured against). */
rflbm_status rflbm_batch_step_separate(rflbm_batch* b, int64_t nsteps);
/* Waits; EUNSTABLE if any replica's instability flag is set. */
rflbm_status rflbm_batch_sync(rflbm_batch* b);
int64_t rflbm_batch_step_count(const rflbm_batch* b);
/* Sets t for every replica (checkpoint restart of a batch).  A change of parity
 * takes one temporary population plane of the largest replica, allocated
 * before any replica moves: ENOMEM leaves the batch unchanged. */
rflbm_status rflbm_batch_set_step_count(rflbm_batch* b, int64_t t);
/* The ensemble statistics of rflbm_stats_config (Sec. III, equilibration
 * ratios) for every replica of the batch: sampled by the batched step on every
 * step whose count t is a multiple of `every` (0: off), before that step's
 * collision, into each replica's own accumulators (read with rflbm_get_stats
 * on its view).  Per-tile FP64 partials are summed in a fixed order, so the
 * sums are reproducible bit for bit for a given tile size (which sets that
 * order); across tile sizes, and against a stand-alone lattice, they agree to
 * FP64 rounding. */
rflbm_status rflbm_batch_stats_config(rflbm_batch* b, int32_t every);
/* Total nodes over all replicas. */
int64_t rflbm_batch_nodes(const rflbm_batch* b);
/* Launch shape: tile = nodes per work item (128 or 256, one thread per node),
 * blocks_per_cu = size of the persistent grid per compute unit (0: one block
 * per tile), graph_steps = steps per captured hipGraph (even, 0 = no graph).
 * Results do not depend on the shape. */
rflbm_status rflbm_batch_set_launch(rflbm_batch* b, int32_t tile, int32_t blocks_per_cu,
                                    int32_t graph_steps);
rflbm_status rflbm_batch_get_launch(const rflbm_batch* b, int32_t* tile, int32_t* blocks_per_cu,
                                    int32_t* graph_steps);
/* Times nsteps batch steps with HIP events on the batch stream. */
rflbm_status rflbm_batch_time_steps(rflbm_batch* b, int64_t nsteps, double* ms);
/* Picks the fastest launch shape by timing trial_steps (even) steps of each
 * candidate (tile 128/256 x blocks per CU 0/2/4/8/16).  The trials run on the
 * batch's own state, which is copied aside first (device memory for one copy
 * of every replica region, ENOMEM if that is not available) and restored with
 * the step count afterwards, so the simulation continues bit for bit as if
 * untuned.  With a cache_path (text file, one line per batch signature:
 * device, storage, rounds, replica boxes), a cached choice is applied without
 * timing and new choices are appended.  The graph length is kept. */
rflbm_status rflbm_batch_autotune(rflbm_batch* b, int32_t trial_steps, const char* cache_path);

/* Diagnostics.
 * rflbm_rng_normals: for count nodes n = node0 .. node0 + count - 1 at step t,
 * writes the 24 uniforms (FP32, radius and angle uniforms as above) and the
 * 24 normals (FP32) the step
 * kernel draws, to device arrays u[24 * count] and z[24 * count] (node-major).
 * rflbm_copy: a plain device-to-device copy kernel of `bytes` bytes (multiple
 * of 16, both pointers 16-byte aligned) on hip_stream, the reference for
 * achievable HBM bandwidth. */
rflbm_status rflbm_rng_normals(uint64_t seed, uint32_t stream_id, uint32_t rounds, uint32_t node0,
                               uint32_t count, uint32_t t, float* u, float* z, void* hip_stream);
rflbm_status rflbm_copy(void* dst, const void* src, size_t bytes, void* hip_stream);

/* Text of the last failure on the calling thread ("" if none). */
const char* rflbm_last_error(void);
/* Library version string. */
const char* rflbm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RFLBM_H */
