/*
 * rflbm_oracle.c -- plain, slow, FP64 CPU oracle of the regularized fluctuating
 * lattice Boltzmann update (Reg-FLBM) on the D3Q27 lattice, after Lauricella,
 * Montessori, Tiribocchi and Succi, "Regularized Fluctuating Lattice Boltzmann
 * Model" (arXiv:2507.08820).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the GPU
 * path is checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header, table
 * or constant generator with the GPU library, and the GPU library never loads it.
 *
 * Form.  Everything is written the way the paper states it, with no blocking,
 * factorisation or fusion:
 *   - the 27 velocities and weights of Table I;
 *   - the 27 Hermite polynomials of Table II, typed in from the table's
 *     polynomial column, and the dense 27x27 matrix M_ki = e_ki they give;
 *   - the normalisation b_k = sum_i w_i e_ki^2 (Eq. normal_fact);
 *   - macroscopic density and momentum (Eqs. eq:rho, eq:u);
 *   - the equilibrium Hermite coefficients by the recursion
 *     a0^(n) = a0^(n-1) u (Eq. rec-eq) along each mode's Hermite index string,
 *     and f^(0) from the full Hermite sum (Eq. hermite_feq2);
 *   - the non-equilibrium Hermite coefficients a1 = sum_i (f_i - f_i^(0)) H_i
 *     (Eq. hermitcoeffneq) and f^(1,h) from Eq. hermite_fneq2h;
 *   - the noise amplitude phi_k of Eq. fluct_phi and the noise term
 *     w_i sum_{k=4}^{26} b_k^-1 e_ki phi_k r_k of Eq. r-flbe2;
 *   - the post-collision population of Eq. r-flbe2 (Reg-FLBM) or Eq. flbe
 *     (BGK-FLBM comparator, equilibrium from Eq. hermite_feq2 as in Sec. III);
 *   - optionally (model 2) the ghost non-equilibrium coefficients of orders
 *     3..6 rebuilt from the second-order ones and u by the recursion of
 *     Eq. recursive_eq, relaxed with omega_g as in Eq. r-flbe with the split
 *     f^(1) = f^(1,h) + f^(1,g) of Sec. II.B;
 *   - push streaming f_i(x + c_i, t + 1) = f*_i(x, t) (Eq. eq:streaming) on a
 *     periodic box;
 *   - an optional thermalised start drawn from the stationary covariance
 *     rho0 kT w_i / c_s^2 (ora_init_thermal).
 *
 * Readings where the paper is silent (they are listed with their reasons in the
 * design notes of the repository):
 *   - the density inside phi_k is the local density of the node;
 *   - separate bulk and shear rates act on the trace and deviator of the
 *     diagonal second-order block {xx, yy, zz} for both relaxation and noise;
 *     with equal rates this is exactly Eq. r-flbe2;
 *   - ghost modes (k >= 10) relax from their projected non-equilibrium
 *     coefficient by (1 - omega_g,k) with noise amplitude phi_k(omega_g,k);
 *     at the paper's omega_g = 1 the relaxed part vanishes as in Eq. r-flbe2;
 *     model 2 relaxes instead the coefficient that Eq. recursive_eq rebuilds
 *     (same noise); "perm(alpha_n)" is read as the sum over the n - 1 ways of
 *     pairing alpha_n with one of the first n - 1 indices (the cyclic
 *     permutations of those indices), the original term included;
 *   - the random numbers: Philox4x32-R (Salmon, Moraes, Dror and Shaw, SC'11,
 *     "Parallel random numbers: as easy as 1, 2, 3") with key (seed low word,
 *     seed high word) and counter (node, step, call j = 0..3, stream id).
 *     The four words w0..w3 of call j give three Box-Muller pairs p = 3j + m:
 *     radius uniforms from the top 23 bits b = w_m >> 9 of w0, w1, w2,
 *     U_2p = 1 - b 2^-23 in [2^-23, 1]; angle uniforms from 16 bits a,
 *     U_2p+1 = a 2^-16 in [0, 1), with a = w3 >> 16 (m = 0), w3 & 0xFFFF
 *     (m = 1) and (w0 & 0xFF) 2^8 + (w1 & 0xFF) (m = 2), bits the radii do
 *     not use; all held exactly in single precision.  The Box-Muller
 *     transform of (U_2p, U_2p+1) gives z_2p = R cos(theta), z_2p+1 =
 *     R sin(theta), R = sqrt(-2 ln U_2p), theta = 2 pi U_2p+1; mode k (4..26)
 *     receives r_k = z_(k-4); z_23 is unused.  (16 angle bits are plenty:
 *     the variance of R cos(theta) over a grid of 2^16 angles is exact; the
 *     radius keeps 23 bits because its smallest uniform sets the tail, here
 *     at 5.65 standard deviations.)
 *
 * Pins.  The Philox bit stream is pinned to the published definition of the
 * round by inversion: the tests undo R rounds of that definition (its odd
 * multipliers are invertible mod 2^32) and must recover every counter.  The
 * uniforms and normals are pinned statistically and by their documented
 * layout.  Every other function is pinned by the tests against values printed
 * in the paper and closed forms.
 *
 * Layout of a lattice in this file: f[i * N + n], i the canonical population
 * index (c = (i % 3 - 1, (i / 3) % 3 - 1, i / 9 - 1)), n = x + nx (y + ny z).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NPOP 27
#define NMODE 27

static const double CS2 = 1.0 / 3.0; /* lattice speed of sound squared (Sec. II.A) */

/* --------------------------------------------------------------------------
 * Table I: velocities and weights.  Population i has velocity
 * (i % 3 - 1, (i / 3) % 3 - 1, i / 9 - 1); its weight is fixed by |c_i|^2.
 * ------------------------------------------------------------------------ */
static void velocity(int i, int c[3]) {
  c[0] = i % 3 - 1;
  c[1] = (i / 3) % 3 - 1;
  c[2] = i / 9 - 1;
}

static double weight(int i) {
  int c[3];
  velocity(i, c);
  int c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
  switch (c2) {
    case 0: return 8.0 / 27.0;
    case 1: return 2.0 / 27.0;
    case 2: return 1.0 / 54.0;
    default: return 1.0 / 216.0;
  }
}

/* --------------------------------------------------------------------------
 * Table II: Hermite basis.  e_ki is the polynomial of column "e_ki", typed in
 * as printed.  n_k is the order, mu_k the multiplicity, and herm_index[k] the
 * subscript of the Hermite symbol H^(n)_{...} (used by the recursion of
 * Eq. rec-eq).
 * ------------------------------------------------------------------------ */
static const int herm_order[NMODE] = {0, 1, 1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3,
                                      3, 3, 3, 4, 4, 4, 4, 4, 4, 5, 5, 5, 6};
static const int herm_mult[NMODE] = {1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 3, 3, 3, 3,
                                     3, 3, 6, 6, 6, 6, 12, 12, 12, 30, 30, 30, 90};
static const char* const herm_index[NMODE] = {
    "",     "x",     "y",     "z",     "xx",    "yy",    "zz",
    "xy",   "xz",    "yz",    "xxy",   "xxz",   "xyy",   "xzz",
    "yzz",  "yyz",   "xyz",   "xxyy",  "xxzz",  "yyzz",  "xyzz",
    "xyyz", "xxyz",  "xxyzz", "xxyyz", "xyyzz", "xxyyzz"};

static double herm_poly(int k, const int ci[3]) {
  const double x = ci[0], y = ci[1], z = ci[2], s = CS2;
  switch (k) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * x - s;
    case 5: return y * y - s;
    case 6: return z * z - s;
    case 7: return x * y;
    case 8: return x * z;
    case 9: return y * z;
    case 10: return x * x * y - s * y;
    case 11: return x * x * z - s * z;
    case 12: return x * y * y - s * x;
    case 13: return x * z * z - s * x;
    case 14: return y * z * z - s * y;
    case 15: return y * y * z - s * z;
    case 16: return x * y * z;
    case 17: return x * x * y * y - s * (x * x + y * y) + s * s;
    case 18: return x * x * z * z - s * (x * x + z * z) + s * s;
    case 19: return y * y * z * z - s * (y * y + z * z) + s * s;
    case 20: return x * y * z * z - s * x * y;
    case 21: return x * y * y * z - s * x * z;
    case 22: return x * x * y * z - s * y * z;
    case 23: return x * x * y * z * z - s * (x * x * y + y * z * z) + s * s * y;
    case 24: return x * x * y * y * z - s * (x * x * z + y * y * z) + s * s * z;
    case 25: return x * y * y * z * z - s * (x * y * y + x * z * z) + s * s * x;
    case 26:
      return x * x * y * y * z * z - s * (x * x * y * y + x * x * z * z + y * y * z * z) +
             s * s * (x * x + y * y + z * z) - s * s * s;
    default: return 0.0;
  }
}

/* Tables built once from the definitions above. */
static double W[NPOP];          /* w_i */
static int C[NPOP][3];          /* c_i */
static double E[NMODE][NPOP];   /* M_ki = e_ki */
static double B[NMODE];         /* b_k = sum_i w_i e_ki^2 (Eq. normal_fact) */
static double HCOEF[NMODE];     /* mu_k / (c_s^(2 n_k) n_k!) (Eq. hermite_feq2) */
static int tables_ready = 0;

static double factorial(int n) {
  double r = 1.0;
  for (int j = 2; j <= n; ++j) r *= j;
  return r;
}

static void build_tables(void) {
  if (tables_ready) return;
  for (int i = 0; i < NPOP; ++i) {
    velocity(i, C[i]);
    W[i] = weight(i);
  }
  for (int k = 0; k < NMODE; ++k) {
    double bk = 0.0;
    for (int i = 0; i < NPOP; ++i) {
      E[k][i] = herm_poly(k, C[i]);
      bk += W[i] * E[k][i] * E[k][i];
    }
    B[k] = bk;
    HCOEF[k] = herm_mult[k] / (pow(CS2, herm_order[k]) * factorial(herm_order[k]));
  }
  tables_ready = 1;
}

/* Exposes the tables so that the tests can pin them to the paper. */
void ora_tables(int32_t* c, double* w, double* e, double* b, double* hcoef, int32_t* order,
                int32_t* mult) {
  build_tables();
  for (int i = 0; i < NPOP; ++i) {
    if (c) for (int a = 0; a < 3; ++a) c[3 * i + a] = C[i][a];
    if (w) w[i] = W[i];
  }
  for (int k = 0; k < NMODE; ++k) {
    if (e) for (int i = 0; i < NPOP; ++i) e[k * NPOP + i] = E[k][i];
    if (b) b[k] = B[k];
    if (hcoef) hcoef[k] = HCOEF[k];
    if (order) order[k] = herm_order[k];
    if (mult) mult[k] = herm_mult[k];
  }
}

/* --------------------------------------------------------------------------
 * Random numbers (the paper does not name its generator).
 * Philox4x32-R from the published description: each round multiplies words 0
 * and 2 by fixed 32-bit constants into 64-bit products; the new word 0 is the
 * high half of the second product xor word 1 xor key 0, word 1 the low half of
 * the second product, word 2 the high half of the first product xor word 3 xor
 * key 1, word 3 the low half of the first product.  Between rounds the key
 * words are advanced by the Weyl constants (golden ratio and sqrt(3) - 1 in
 * 32-bit fixed point).
 * ------------------------------------------------------------------------ */
#define PHILOX_MUL_A 0xD2511F53u
#define PHILOX_MUL_B 0xCD9E8D57u
#define PHILOX_WEYL_A 0x9E3779B9u
#define PHILOX_WEYL_B 0xBB67AE85u

void ora_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t rounds,
                    uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (uint32_t r = 0; r < rounds; ++r) {
    if (r > 0) {
      k0 += PHILOX_WEYL_A;
      k1 += PHILOX_WEYL_B;
    }
    uint64_t pa = (uint64_t)PHILOX_MUL_A * (uint64_t)x0;
    uint64_t pb = (uint64_t)PHILOX_MUL_B * (uint64_t)x2;
    uint32_t n0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
    uint32_t n1 = (uint32_t)pb;
    uint32_t n2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
    uint32_t n3 = (uint32_t)pa;
    x0 = n0; x1 = n1; x2 = n2; x3 = n3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniforms 6j .. 6j + 5 (three radius-angle pairs) from the four words of
 * Philox call j, as laid out in the header: radius uniforms 1 - b 2^-23 from
 * the top 23 bits of words 0, 1, 2 (never 0, so the logarithm is finite),
 * angle uniforms a 2^-16 from 16 bits the radii leave unused. */
static void uniforms_of_call(const uint32_t w[4], double u[6]) {
  const uint32_t angle_bits[3] = {w[3] >> 16, w[3] & 0xFFFFu, ((w[0] & 0xFFu) << 8) | (w[1] & 0xFFu)};
  for (int m = 0; m < 3; ++m) {
    u[2 * m] = 1.0 - (double)(w[m] >> 9) / 8388608.0;
    u[2 * m + 1] = (double)angle_bits[m] / 65536.0;
  }
}

/* The 24 uniforms of one (node, step, stream) and their 24 Box-Muller normals.
 * r[k - 4] for k = 4..26 are the 23 normals the update uses. */
void ora_uniforms(uint64_t seed, uint32_t stream_id, uint32_t rounds, uint32_t node, uint32_t step,
                  double u[24]) {
  const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  for (uint32_t j = 0; j < 4; ++j) {
    const uint32_t ctr[4] = {node, step, j, stream_id};
    uint32_t words[4];
    ora_philox4x32(ctr, key, rounds, words);
    uniforms_of_call(words, u + 6 * j);
  }
}

void ora_normals(uint64_t seed, uint32_t stream_id, uint32_t rounds, uint32_t node, uint32_t step,
                 double z[24]) {
  double u[24];
  ora_uniforms(seed, stream_id, rounds, node, step, u);
  const double two_pi = 2.0 * 3.14159265358979323846;
  for (int p = 0; p < 12; ++p) {
    double radius = sqrt(-2.0 * log(u[2 * p]));
    double theta = two_pi * u[2 * p + 1];
    z[2 * p] = radius * cos(theta);
    z[2 * p + 1] = radius * sin(theta);
  }
}

/* --------------------------------------------------------------------------
 * Equilibrium (Eqs. eq:rho, eq:u, rec-eq, hermite_feq2).
 * ------------------------------------------------------------------------ */
static int axis_of(char ch) { return ch == 'x' ? 0 : (ch == 'y' ? 1 : 2); }

/* a0 of mode k: rho followed by one factor u_alpha per index of H_k (Eq. rec-eq). */
static double a0_coefficient(int k, double rho, const double u[3]) {
  double a = rho;
  for (const char* p = herm_index[k]; *p; ++p) a *= u[axis_of(*p)];
  return a;
}

/* Eq. recursive_eq: non-equilibrium coefficient a1^(n) of the first n indices
 * of the Hermite index string s (n >= 2), from the second-order coefficients
 * a2[alpha][beta] and the velocity u:
 *   a1^(n)_{s1..sn} = a1^(n-1)_{s1..s(n-1)} u_sn
 *                     + sum_{j < n} a2_{sj sn} prod_{l < n, l != j} u_sl,
 * where the sum runs over the cyclic permutations of the first n - 1 indices
 * (each of them takes the place next to s_n once). */
static double a1_recursive(const char* s, int n, const double a2[3][3], const double u[3]) {
  if (n == 2) return a2[axis_of(s[0])][axis_of(s[1])];
  const int last = axis_of(s[n - 1]);
  double r = a1_recursive(s, n - 1, a2, u) * u[last];
  for (int j = 0; j < n - 1; ++j) {
    double term = a2[axis_of(s[j])][last];
    for (int l = 0; l < n - 1; ++l)
      if (l != j) term *= u[axis_of(s[l])];
    r += term;
  }
  return r;
}

/* The recursive ghost coefficients of every mode k = 10..26 (out[k]; out[0..9]
 * are set to 0) from the six second-order coefficients a2 in Table II order
 * (xx, yy, zz, xy, xz, yz) and u.  Exposed for the tests. */
void ora_ghost_recursive(const double a2v[6], const double u[3], double out[NMODE]) {
  const double a2[3][3] = {{a2v[0], a2v[3], a2v[4]}, {a2v[3], a2v[1], a2v[5]}, {a2v[4], a2v[5], a2v[2]}};
  for (int k = 0; k < NMODE; ++k)
    out[k] = k < 10 ? 0.0 : a1_recursive(herm_index[k], herm_order[k], a2, u);
}

void ora_equilibrium(double rho, const double u[3], double feq[NPOP]) {
  build_tables();
  double a0[NMODE];
  for (int k = 0; k < NMODE; ++k) a0[k] = a0_coefficient(k, rho, u);
  for (int i = 0; i < NPOP; ++i) {
    double s = 0.0;
    for (int k = 0; k < NMODE; ++k) s += HCOEF[k] * a0[k] * E[k][i];
    feq[i] = W[i] * s;
  }
}

/* --------------------------------------------------------------------------
 * Collision of one node.
 * ------------------------------------------------------------------------ */
typedef struct {
  double rho0;          /* reference density (storage offsets only; unused here) */
  double kT;            /* k_B T >= 0 */
  double tau_shear;     /* 1 / omega_h on the deviatoric second-order modes */
  double tau_bulk;      /* 1 / omega on the trace of the second-order block */
  double tau_ghost[17]; /* 1 / omega_g,k for k = 10..26 */
  uint64_t seed;
  uint32_t stream_id;
  uint32_t rounds;
  int32_t model;        /* 0: Reg-FLBM (Eq. r-flbe2), 1: BGK-FLBM (Eq. flbe),
                           2: Reg-FLBM with recursive ghosts (Eq. recursive_eq) */
  int32_t pad;
} ora_params;

static double fdt_factor(double omega) { return sqrt(omega * (2.0 - omega)); }

/* f -> post-collision f* given the 23 normals r[k - 4], k = 4..26. */
void ora_collide(const ora_params* p, const double f[NPOP], const double r[23], double fout[NPOP]) {
  build_tables();
  /* Eqs. eq:rho and eq:u */
  double rho = 0.0, ju[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < NPOP; ++i) {
    rho += f[i];
    for (int a = 0; a < 3; ++a) ju[a] += f[i] * C[i][a];
  }
  const double u[3] = {ju[0] / rho, ju[1] / rho, ju[2] / rho};

  /* Eq. hermite_feq2 with Eq. rec-eq */
  double f0[NPOP];
  ora_equilibrium(rho, u, f0);

  /* Noise amplitudes, Eq. fluct_phi with the local density: phi_k^2 =
   * rho kT omega_k (2 - omega_k) b_k / c_s^2.  The square root of the
   * omega-independent part is sqrt(mu b_k), mu = rho kT / c_s^2. */
  const double mu = rho * p->kT / CS2;
  double noise_mode[NMODE];
  for (int k = 0; k < NMODE; ++k) noise_mode[k] = 0.0;

  double relaxed[NMODE]; /* relaxed non-equilibrium Hermite coefficients */
  for (int k = 0; k < NMODE; ++k) relaxed[k] = 0.0;

  if (p->model == 1) {
    /* BGK-FLBM, Eq. flbe: one omega on the whole non-equilibrium part and in
     * every noise amplitude. */
    const double omega = 1.0 / p->tau_shear;
    for (int k = 4; k < NMODE; ++k) noise_mode[k] = sqrt(mu * B[k]) * fdt_factor(omega) * r[k - 4];
    for (int i = 0; i < NPOP; ++i) {
      double noise = 0.0;
      for (int k = 4; k < NMODE; ++k) noise += E[k][i] * noise_mode[k] / B[k];
      fout[i] = f0[i] + (1.0 - omega) * (f[i] - f0[i]) + W[i] * noise;
    }
    return;
  }

  /* Eq. hermitcoeffneq: a1 = sum_i (f_i - f_i^(0)) H_i, k = 4..26. */
  double a1[NMODE];
  for (int k = 0; k < NMODE; ++k) {
    double s = 0.0;
    if (k >= 4)
      for (int i = 0; i < NPOP; ++i) s += (f[i] - f0[i]) * E[k][i];
    a1[k] = s;
  }

  const double om_s = 1.0 / p->tau_shear, om_b = 1.0 / p->tau_bulk;
  /* Diagonal block {xx, yy, zz}: trace part relaxes with omega_b, deviator
   * with omega_s; the noise is split the same way.  With omega_b = omega_s
   * this is (1 - omega_h) a1 and phi_k r_k exactly. */
  const double a_mean = (a1[4] + a1[5] + a1[6]) / 3.0;
  const double r_mean = (r[0] + r[1] + r[2]) / 3.0;
  for (int k = 4; k <= 6; ++k) {
    relaxed[k] = (1.0 - om_b) * a_mean + (1.0 - om_s) * (a1[k] - a_mean);
    noise_mode[k] =
        sqrt(mu * B[k]) * (fdt_factor(om_b) * r_mean + fdt_factor(om_s) * (r[k - 4] - r_mean));
  }
  for (int k = 7; k <= 9; ++k) {
    relaxed[k] = (1.0 - om_s) * a1[k];
    noise_mode[k] = sqrt(mu * B[k]) * fdt_factor(om_s) * r[k - 4];
  }
  /* Ghosts: the projected coefficient a1 (model 0), or the one Eq.
   * recursive_eq rebuilds from the unrelaxed second-order a1 and u (model 2). */
  double ghost_neq[NMODE];
  if (p->model == 2) {
    const double a2v[6] = {a1[4], a1[5], a1[6], a1[7], a1[8], a1[9]};
    ora_ghost_recursive(a2v, u, ghost_neq);
  } else {
    for (int k = 0; k < NMODE; ++k) ghost_neq[k] = a1[k];
  }
  for (int k = 10; k < NMODE; ++k) {
    const double om_g = 1.0 / p->tau_ghost[k - 10];
    relaxed[k] = (1.0 - om_g) * ghost_neq[k];
    noise_mode[k] = sqrt(mu * B[k]) * fdt_factor(om_g) * r[k - 4];
  }

  /* Eq. r-flbe2: f* = f^(0) + relaxed f^(1,h) (+ relaxed ghost part, zero at
   * omega_g = 1) + w_i sum_{k>=4} b_k^-1 e_ki phi_k r_k.  The relaxed
   * f^(1,h) is Eq. hermite_fneq2h with the relaxed coefficients. */
  for (int i = 0; i < NPOP; ++i) {
    double fneq_h = 0.0, fneq_g = 0.0, noise = 0.0;
    for (int k = 4; k <= 9; ++k) fneq_h += HCOEF[k] * relaxed[k] * E[k][i];
    for (int k = 10; k < NMODE; ++k) fneq_g += HCOEF[k] * relaxed[k] * E[k][i];
    for (int k = 4; k < NMODE; ++k) noise += E[k][i] * noise_mode[k] / B[k];
    fout[i] = f0[i] + W[i] * fneq_h + W[i] * fneq_g + W[i] * noise;
  }
}

/* --------------------------------------------------------------------------
 * Whole-lattice step: collide every node with its own normals, then push
 * f*_i(x) to x + c_i (Eq. eq:streaming), periodic in every direction.
 * ------------------------------------------------------------------------ */
static void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

int ora_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int ora_step(const ora_params* p, int32_t nx, int32_t ny, int32_t nz, uint32_t step,
             const double* f, double* fnew, int32_t nthreads) {
  if (nx < 1 || ny < 1 || nz < 1 || !p || !f || !fnew) return -1;
  build_tables();
  set_threads(nthreads);
  const int64_t N = (int64_t)nx * ny * nz;
  const int noisy = p->kT > 0.0;
#pragma omp parallel for schedule(static)
  for (int64_t row = 0; row < (int64_t)ny * nz; ++row) {
    const int32_t y = (int32_t)(row % ny), z = (int32_t)(row / ny);
    for (int32_t x = 0; x < nx; ++x) {
      const int64_t n = x + (int64_t)nx * (y + (int64_t)ny * z);
      double fl[NPOP], fs[NPOP], z24[24];
      for (int i = 0; i < NPOP; ++i) fl[i] = f[i * N + n];
      if (noisy)
        ora_normals(p->seed, p->stream_id, p->rounds, (uint32_t)n, step, z24);
      else
        for (int q = 0; q < 24; ++q) z24[q] = 0.0;
      ora_collide(p, fl, z24, fs);
      for (int i = 0; i < NPOP; ++i) {
        const int32_t xd = (x + C[i][0] + nx) % nx;
        const int32_t yd = (y + C[i][1] + ny) % ny;
        const int32_t zd = (z + C[i][2] + nz) % nz;
        fnew[i * N + xd + (int64_t)nx * (yd + (int64_t)ny * zd)] = fs[i];
      }
    }
  }
  return 0;
}

/* nsteps steps starting at step counter step0; f holds the state in and out,
 * work is caller scratch of the same size. */
int ora_run(const ora_params* p, int32_t nx, int32_t ny, int32_t nz, uint32_t step0,
            int32_t nsteps, double* f, double* work, int32_t nthreads) {
  const int64_t total = (int64_t)NPOP * nx * ny * nz;
  double* a = f;
  double* b = work;
  for (int32_t s = 0; s < nsteps; ++s) {
    int rc = ora_step(p, nx, ny, nz, step0 + (uint32_t)s, a, b, nthreads);
    if (rc) return rc;
    double* t = a; a = b; b = t;
  }
  if (a != f) memcpy(f, a, (size_t)total * sizeof(double));
  return 0;
}

/* Thermalised start: f_i = f^(0)_i(rho, u) + sqrt(mu w_i) xi_i with
 * mu = rho0 kT / c_s^2, the stationary covariance mu w_i delta_ij that the
 * fluctuation-dissipation balance of Eq. fluct_phi sustains in the linear
 * regime.  xi_i is the i-th normal of the node's Box-Muller stream drawn at the
 * reserved step word 0xFFFFFFFF with calls j = 0..4 (30 normals, 27 used):
 * call j gives uniforms 6j .. 6j + 5 as in ora_uniforms. */
int ora_init_thermal(const ora_params* p, int32_t nx, int32_t ny, int32_t nz, const double* rho,
                     const double* u, double* f) {
  build_tables();
  const int64_t N = (int64_t)nx * ny * nz;
  const uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), (uint32_t)(p->seed >> 32)};
  const double mu = p->rho0 * p->kT / CS2;
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n) {
    double fe[NPOP], uni[30], z[30];
    const double un[3] = {u ? u[n] : 0.0, u ? u[N + n] : 0.0, u ? u[2 * N + n] : 0.0};
    ora_equilibrium(rho ? rho[n] : p->rho0, un, fe);
    for (uint32_t j = 0; j < 5; ++j) {
      const uint32_t ctr[4] = {(uint32_t)n, 0xFFFFFFFFu, j, p->stream_id};
      uint32_t words[4];
      ora_philox4x32(ctr, key, p->rounds, words);
      uniforms_of_call(words, uni + 6 * j);
    }
    for (int q = 0; q < 15; ++q) {
      const double radius = sqrt(-2.0 * log(uni[2 * q]));
      const double theta = 2.0 * 3.14159265358979323846 * uni[2 * q + 1];
      z[2 * q] = radius * cos(theta);
      z[2 * q + 1] = radius * sin(theta);
    }
    for (int i = 0; i < NPOP; ++i) f[i * N + n] = fe[i] + sqrt(mu * W[i]) * z[i];
  }
  return 0;
}

/* Equilibrium populations for given rho and u fields (SoA: u[a * N + n]). */
int ora_init_equilibrium(int32_t nx, int32_t ny, int32_t nz, const double* rho, const double* u,
                         double* f) {
  build_tables();
  const int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n) {
    double fe[NPOP];
    const double un[3] = {u[n], u[N + n], u[2 * N + n]};
    ora_equilibrium(rho[n], un, fe);
    for (int i = 0; i < NPOP; ++i) f[i * N + n] = fe[i];
  }
  return 0;
}
