/*
 * Oracle for the 1D pair-cascade PIC step -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain scalar C, built with -O2 -ffp-contract=off so that every product
 * and sum is rounded on its own (no fused multiply-add).  Only the tests,
 * the smoke check and the benchmark's CPU-baseline leg use it.  It shares
 * nothing with the HIP library.
 *
 * What it computes (arXiv:2012.05587):
 *   - section 2: every lepton whose Lorentz factor reaches gamma_thr emits a
 *     pair of combined energy gamma_pair = f*gamma_thr, split equally between
 *     the electron and the positron;
 *   - section 3, population bookkeeping: the emitter keeps its direction and
 *     drops by gamma_pair per emission, into [gamma_thr - gamma_pair, gamma_thr];
 *   - section 3, Eq. 4: Ampere's law, dE/dt = -J in normalised units.
 * The paper makes pair production in place (zero photon mean free path);
 * l_gamma > 0 adds a photon that streams at c and converts after an
 * exponentially distributed path of mean l_gamma cells (its section 2
 * motivates the finite path through the growth of chi_gamma with distance).
 *
 * Readings where the paper is silent (it names its PIC code but gives no
 * scheme): cloud-in-cell charge on the nodes x = c*dx, E and J at cell
 * centres; gather by averaging E to the nodes and interpolating linearly;
 * exact charge-conserving flux J*dt = sum q*w*(offset change) per cell
 * crossed; seeded momenta are p at t = -dt/2; emission is tested on
 * gamma(p^{n+1/2}) at the post-move position; k emissions in one step are
 * taken by repeated subtraction; secondaries move along the emitter's
 * direction.  Positions are a cell index plus an offset on a fixed grid of
 * 2^-K cells (K = 40 in binary64, 24 in binary32), and the flux is summed in
 * int64 units of 2^-K, so the deposit is exact and independent of the order
 * in which particles are visited.
 *
 * Precision: in ORC_FP64 every per-particle quantity is binary64.  In
 * ORC_MIXED every per-particle operation is rounded to binary32 (rounding a
 * binary64 result of +,-,*,/,sqrt of binary32 operands to binary32 gives the
 * correctly rounded binary32 result); the field, the Ampere update and the
 * diagnostics stay binary64.
 */
#include "pic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_TAG_SEED   1u
#define ORC_TAG_PHOTON 2u
#define ORC_TAG_THRESHOLD 3u
#define ORC_MAX_EMIT   64

typedef struct {
  int32_t*  cell;
  int64_t*  offq;   /* offset in units of 2^-K of a cell, in [0, 2^K) */
  double*   p;      /* momentum in m c (binary32 values in mixed mode) */
  uint64_t* id;
  int64_t   n, cap;
} orc_species;

typedef struct {
  int64_t  xq;        /* conversion point, units of 2^-K cells from x = 0 */
  int64_t  conv_step; /* converts at the end of this step */
  int32_t  dir;
  uint64_t child;     /* id of the electron; the positron is child | 1 */
} orc_photon;

struct orc_gap {
  orc_params   prm;
  int          mixed;
  int          K;
  int64_t      one;        /* 2^K */
  orc_species  sp[2];      /* 0: electrons (q = -1), 1: positrons (q = +1) */
  orc_photon*  ph;
  int64_t      n_ph, cap_ph;
  double*      E;
  int64_t*     F;          /* flux of the last step, units of w * 2^-K */
  uint32_t*    table;
  int64_t      table_len;
  int64_t      step;
  int          status;
  orc_history_row* hist;
  int64_t      n_hist, cap_hist;
  /* cumulative tallies */
  int64_t      pairs_created, photons_emitted, photons_escaped, absorbed[2];
  double       lost_energy;
  /* pair-event map (the (x, t) map of section 7's figure): pairs made at step
   * n in cell c count in row (n / ev_steps) % ev_rows, column c * ev_x / N_c */
  int64_t*     ev_map;
  int32_t      ev_x, ev_steps, ev_rows;
};

/* ------------------------------------------------------------------------ */
/* Philox4x64-10: Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3" (SC'11).  Each round multiplies two counter words by the
 * round multipliers, swaps and xors with the key; the key is bumped by the
 * Weyl constants between rounds.                                            */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  unsigned __int128 prod = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(prod >> 64);
  *lo = (uint64_t)prod;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c0, &hi0, &lo0);
    mulhilo64(M1, c2, &hi1, &lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    uint64_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Philox4x32-10 (same paper): the 32-bit form, with 32x32 -> 64-bit
 * products, its own round multipliers and Weyl constants; four 32-bit
 * counter words, two key words. */
static void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  uint64_t prod = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(prod >> 32);
  *lo = (uint32_t)prod;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo32(M0, c0, &hi0, &lo0);
    mulhilo32(M1, c2, &hi1, &lo1);
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The seeding draw of pair i: Philox4x64-10, key (i, seed), counter
 * (0, 0, 1, 0). */
static void draw_seed(uint64_t i, uint64_t seed, uint64_t out[4]) {
  uint64_t ctr[4] = {0, 0, ORC_TAG_SEED, 0};
  uint64_t key[2] = {i, seed};
  orc_philox4x64_10(ctr, key, out);
}

/* A draw of lepton `id` during the run (tag 2: emission j at step n; tag 3:
 * its threshold, n = j = 0): Philox4x32-10, key (seed low, seed high),
 * counter (n, j | tag << 8, id low, id high).  Words 0 and 1 form the 64-bit
 * value `bits`, word 2 is `u32`. */
static void draw_run(uint64_t id, uint64_t seed, uint64_t step, uint64_t j, uint32_t tag,
                     uint64_t* bits, uint32_t* u32) {
  uint32_t ctr[4] = {(uint32_t)step, (uint32_t)j | (tag << 8), (uint32_t)id, (uint32_t)(id >> 32)};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  *bits = ((uint64_t)out[1] << 32) | out[0];
  *u32 = out[2];
}

/* Photon path, discretised to whole steps.  A photon streams c*dt/dx cells
 * per step; with an exponential path of mean l_gamma cells the probability of
 * still being in flight after k steps is q^k, q = exp(-c dt / (l_gamma dx)).
 * T_k = floor(q^k 2^32); the draw u (32 bits) converts at
 * n_conv = min{k >= 1 : u >= T_k}, so P(n_conv > k) = T_k / 2^32.
 * Returns the number of entries (T_0 .. T_{len-1}, with T_{len-1} = 0).   */
int64_t orc_conv_table(double dt, double dx, double l_gamma, uint32_t* table, int64_t max_len) {
  if (!(l_gamma > 0.0)) return 0;
  double r = dt / (l_gamma * dx);
  int64_t k = 0;
  for (;;) {
    double t = floor(ldexp(exp(-((double)k * r)), 32));
    uint64_t tk = t >= 4294967296.0 ? 4294967296ull : (uint64_t)t;
    if (table) {
      if (k >= max_len) return -1;
      table[k] = tk >= 4294967296ull ? 0xFFFFFFFFu : (uint32_t)tk;
    }
    ++k;
    if (tk == 0) break;
  }
  return k;
}

static int64_t conv_steps(const orc_gap* g, uint32_t u) {
  /* the definition, scanned from k = 1 (T_0 = 2^32 is never reached) */
  for (int64_t k = 1; k < g->table_len; ++k)
    if ((uint64_t)u >= (uint64_t)g->table[k]) return k;
  return g->table_len - 1;
}

/* ------------------------------------------------------------------------ */
static double R(const orc_gap* g, double x) { return g->mixed ? (double)(float)x : x; }

/* Energy diagnostics stay binary64 in both precisions: a lepton's Lorentz
 * factor is re-evaluated in binary64 from its stored momentum (a binary32
 * value in mixed precision), not taken from the push's binary32 gamma. */
static double gamma64(double p) { return sqrt(1.0 + p * p); }

/* Emission threshold of lepton `id` under a spread sigma of gamma_thr: a
 * fixed property of the lepton, uniform in gamma_thr (1 - sigma, 1 + sigma).
 * u = (top 53 bits of the 64-bit value of its tag-3 draw) / 2^53, then
 * gamma_thr (1 + sigma (2u - 1)) in binary64, one rounding per operation,
 * rounded to the particle precision at the end. */
static double lepton_threshold(const orc_gap* g, uint64_t id) {
  uint64_t bits;
  uint32_t u32;
  draw_run(id, g->prm.seed, 0, 0, ORC_TAG_THRESHOLD, &bits, &u32);
  const double x = ldexp((double)(bits >> 11), -53);
  const double a = 2.0 * x - 1.0;
  const double t = g->prm.gamma_thr * (1.0 + g->prm.gamma_thr_spread * a);
  return R(g, t);
}

int orc_validate(const orc_params* p) {
  if (!p) return ORC_ERR_ARG;
  if (p->n_cells < 2) return ORC_ERR_ARG;
  if (!(p->dx > 0.0) || !(p->dt > 0.0) || !(p->dt < p->dx)) return ORC_ERR_ARG;
  if (p->boundary != ORC_BC_PERIODIC && p->boundary != ORC_BC_ABSORBING) return ORC_ERR_ARG;
  if (!isfinite(p->e0)) return ORC_ERR_ARG;
  if (!(p->gamma_thr > 1.0) || !(p->f > 0.0) || !(p->f < 1.0)) return ORC_ERR_ARG;
  if (isfinite(p->gamma_thr)) {
    if (!(p->f * p->gamma_thr >= 2.0)) return ORC_ERR_ARG;           /* secondaries have gamma >= 1 */
    if (!((1.0 - p->f) * p->gamma_thr >= 1.0)) return ORC_ERR_ARG;  /* emitter keeps gamma >= 1 */
  }
  if (!(p->l_gamma >= 0.0) || !isfinite(p->l_gamma)) return ORC_ERR_ARG;
  if (!(p->weight >= 0.0) || !isfinite(p->weight)) return ORC_ERR_ARG;
  if (!isfinite(p->j_m)) return ORC_ERR_ARG;
  if (!(p->gamma_thr_spread >= 0.0) || !(p->gamma_thr_spread < 1.0)) return ORC_ERR_ARG;
  /* the lowest threshold still leaves the emitter gamma >= 1 after an emission */
  if (p->gamma_thr_spread > 0.0 && isfinite(p->gamma_thr) &&
      !((1.0 - p->f - p->gamma_thr_spread) * p->gamma_thr >= 1.0))
    return ORC_ERR_ARG;
  if (p->shape != ORC_SHAPE_LINEAR && p->shape != ORC_SHAPE_QUADRATIC) return ORC_ERR_ARG;
  if (p->shape == ORC_SHAPE_QUADRATIC && p->n_cells < 4) return ORC_ERR_ARG;
  if (p->precision != ORC_FP64 && p->precision != ORC_MIXED) return ORC_ERR_ARG;
  if (p->capacity < 0) return ORC_ERR_ARG;
  /* Positions are int64 multiples of 2^-K cells.  The domain and a photon's
   * longest path stay below 2^62 of them.  The conversion table ends after
   * at most ceil(32 ln 2 / r) + 3 entries, r = dt / (l_gamma dx), and a
   * photon moves dt/dx cells per step. */
  {
    const double unit = ldexp(1.0, p->precision == ORC_MIXED ? 24 : 40);
    if ((double)p->n_cells * unit > 0x1p62) return ORC_ERR_ARG;
    if (p->l_gamma > 0.0) {
      const double r = p->dt / (p->l_gamma * p->dx);
      const double len = ceil(32.0 * log(2.0) / r) + 3.0;
      if ((len + 1.0) * (p->dt / p->dx * unit + 1.0) >= 0x1p62) return ORC_ERR_ARG;
    }
  }
  return ORC_OK;
}

static void* grow(void* ptr, int64_t* cap, int64_t need, size_t elem) {
  if (need <= *cap) return ptr;
  int64_t nc = *cap > 0 ? *cap : 64;
  while (nc < need) nc *= 2;
  void* np = realloc(ptr, (size_t)nc * elem);
  if (!np) abort();
  *cap = nc;
  return np;
}

static void species_reserve(orc_species* s, int64_t need) {
  if (need <= s->cap) return;
  int64_t c0 = s->cap, c1 = s->cap, c2 = s->cap, c3 = s->cap;
  s->cell = (int32_t*)grow(s->cell, &c0, need, sizeof(int32_t));
  s->offq = (int64_t*)grow(s->offq, &c1, need, sizeof(int64_t));
  s->p    = (double*)grow(s->p, &c2, need, sizeof(double));
  s->id   = (uint64_t*)grow(s->id, &c3, need, sizeof(uint64_t));
  s->cap = c0;
}

static void species_push_back(orc_species* s, int32_t cell, int64_t offq, double p, uint64_t id) {
  species_reserve(s, s->n + 1);
  s->cell[s->n] = cell; s->offq[s->n] = offq; s->p[s->n] = p; s->id[s->n] = id;
  s->n++;
}

orc_gap* orc_create(const orc_params* prm) {
  if (orc_validate(prm) != ORC_OK) return NULL;
  orc_gap* g = (orc_gap*)calloc(1, sizeof(orc_gap));
  if (!g) return NULL;
  g->prm = *prm;
  g->mixed = prm->precision == ORC_MIXED;
  g->K = g->mixed ? 24 : 40;
  g->one = (int64_t)1 << g->K;
  g->E = (double*)malloc(sizeof(double) * (size_t)prm->n_cells);
  g->F = (int64_t*)calloc((size_t)prm->n_cells, sizeof(int64_t));
  for (int32_t c = 0; c < prm->n_cells; ++c) g->E[c] = prm->e0;
  g->table_len = orc_conv_table(prm->dt, prm->dx, prm->l_gamma, NULL, 0);
  if (g->table_len > 0) {
    g->table = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)g->table_len);
    orc_conv_table(prm->dt, prm->dx, prm->l_gamma, g->table, g->table_len);
  }
  return g;
}

void orc_destroy(orc_gap* g) {
  if (!g) return;
  for (int s = 0; s < 2; ++s) {
    free(g->sp[s].cell); free(g->sp[s].offq); free(g->sp[s].p); free(g->sp[s].id);
  }
  free(g->ph); free(g->E); free(g->F); free(g->table); free(g->hist); free(g->ev_map);
  free(g);
}

int orc_offset_bits(const orc_gap* g) { return g->K; }

/* Seed plasma (section 3: uniform pair plasma at rest).  Macro-pair i puts an
 * electron (id 2i) and a positron (id 2i+1) at the same point, so the charge
 * density is zero and the uniform initial field satisfies Gauss's law.
 * RANDOM: u = Philox(key (i, seed), counter (0, 0, SEED, 0)); cell from the
 * high 32 bits of u[0] scaled to n_cells, offset from the high 24 bits of
 * u[1].  LATTICE: x_i = (i + 1/2) n_cells / N on the 2^-24 grid.           */
int orc_seed(orc_gap* g, int32_t mode, int64_t n_pairs, int32_t macro_per_pair,
             double p0_minus, double p0_plus) {
  if (!g || n_pairs < 0 || macro_per_pair < 1) return ORC_ERR_ARG;
  if (mode != ORC_SEED_RANDOM && mode != ORC_SEED_LATTICE) return ORC_ERR_ARG;
  if (g->step != 0 || g->sp[0].n != 0 || g->sp[1].n != 0) return ORC_ERR_STATE;
  int64_t N = n_pairs * (int64_t)macro_per_pair;
  if (g->prm.capacity > 0 && N > g->prm.capacity) return ORC_ERR_CAPACITY;
  int shift = g->K - 24;
  double pm = R(g, p0_minus), pp = R(g, p0_plus);
  for (int64_t i = 0; i < N; ++i) {
    int32_t cell;
    int64_t off24;
    if (mode == ORC_SEED_RANDOM) {
      uint64_t u[4];
      draw_seed((uint64_t)i, g->prm.seed, u);
      cell = (int32_t)(((u[0] >> 32) * (uint64_t)g->prm.n_cells) >> 32);
      off24 = (int64_t)(u[1] >> 40);
    } else {
      double x = floor(((double)i + 0.5) * ((double)g->prm.n_cells / (double)N) * 16777216.0);
      int64_t X = (int64_t)x;
      cell = (int32_t)(X >> 24);
      off24 = X & 0xFFFFFF;
    }
    species_push_back(&g->sp[0], cell, off24 << shift, pm, 2u * (uint64_t)i);
    species_push_back(&g->sp[1], cell, off24 << shift, pp, 2u * (uint64_t)i + 1u);
  }
  return ORC_OK;
}

int orc_seed_explicit(orc_gap* g, int32_t species, int64_t n, const int32_t* cell,
                      const double* off, const double* p, const uint64_t* id) {
  if (!g || species < 0 || species > 1 || n < 0) return ORC_ERR_ARG;
  if (g->step != 0) return ORC_ERR_STATE;
  if (g->prm.capacity > 0 && g->sp[species].n + n > g->prm.capacity) return ORC_ERR_CAPACITY;
  for (int64_t i = 0; i < n; ++i) {
    if (cell[i] < 0 || cell[i] >= g->prm.n_cells) return ORC_ERR_ARG;
    if (!(off[i] >= 0.0) || !(off[i] < 1.0) || !isfinite(p[i])) return ORC_ERR_ARG;
  }
  for (int64_t i = 0; i < n; ++i)
    species_push_back(&g->sp[species], cell[i], (int64_t)floor(ldexp(off[i], g->K)),
                      R(g, p[i]), id[i]);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
static int32_t wrap_cell(const orc_gap* g, int32_t c) {
  if (c < 0) return c + g->prm.n_cells;
  if (c >= g->prm.n_cells) return c - g->prm.n_cells;
  return c;
}

/* Quadratic-spline (triangular-shaped cloud) weights of a lepton at X, in
 * units of 2^-K cells from some node.  Its nearest node is j = floor(X/2^K +
 * 1/2) and delta = X/2^K - j lies in [-1/2, 1/2).  The spline gives the
 * nodes j-1, j, j+1 the charge fractions (1/2 - delta)^2 / 2,
 * 3/4 - delta^2, (1/2 + delta)^2 / 2.  As integers in 2^-K: the outer two
 * are rounded down, the middle one takes the rest, so the three sum to 2^K
 * exactly and the deposit built from them conserves charge exactly. */
static void tsc_weights(const orc_gap* g, int64_t X, int64_t* j, int64_t W[3]) {
  const int64_t ONE = g->one, HALF = g->one / 2;
  int64_t jj = (X + HALF) >= 0 ? (X + HALF) / ONE : -((-(X + HALF) + ONE - 1) / ONE);
  const int64_t delta = X - jj * ONE;
  const unsigned __int128 a = (unsigned __int128)(HALF - delta);
  const unsigned __int128 b = (unsigned __int128)(HALF + delta);
  W[0] = (int64_t)((a * a) >> (g->K + 1));
  W[2] = (int64_t)((b * b) >> (g->K + 1));
  W[1] = ONE - W[0] - W[2];
  *j = jj;
}

/* E at cell centre c seen by the gather, with the boundary ghosts:
 * periodic wraps, absorbing repeats the edge value (zero gradient). */
static double e_ghost(const orc_gap* g, int32_t c) {
  if (g->prm.boundary == ORC_BC_PERIODIC) return g->E[wrap_cell(g, c)];
  if (c < 0) return g->E[0];
  if (c >= g->prm.n_cells) return g->E[g->prm.n_cells - 1];
  return g->E[c];
}

static void append_photon(orc_gap* g, int64_t xq, int64_t conv_step, int32_t dir, uint64_t child) {
  g->ph = (orc_photon*)grow(g->ph, &g->cap_ph, g->n_ph + 1, sizeof(orc_photon));
  g->ph[g->n_ph].xq = xq;
  g->ph[g->n_ph].conv_step = conv_step;
  g->ph[g->n_ph].dir = dir;
  g->ph[g->n_ph].child = child;
  g->n_ph++;
}

static void append_pair(orc_gap* g, int64_t n, int32_t cell, int64_t offq, int32_t dir,
                        uint64_t child, double pchild) {
  double p = dir > 0 ? pchild : -pchild;
  species_push_back(&g->sp[0], cell, offq, p, child);
  species_push_back(&g->sp[1], cell, offq, p, child | 1u);
  g->pairs_created++;
  if (g->ev_map) {
    const int64_t row = (n / g->ev_steps) % g->ev_rows;
    const int64_t col = (int64_t)cell * g->ev_x / g->prm.n_cells;
    g->ev_map[row * g->ev_x + col] += 1;
  }
}

int orc_event_map(orc_gap* g, int32_t x_bins, int32_t steps_per_row, int32_t rows) {
  if (!g) return ORC_ERR_ARG;
  free(g->ev_map);
  g->ev_map = NULL;
  if (x_bins == 0) return ORC_OK;
  if (x_bins < 1 || steps_per_row < 1 || rows < 1) return ORC_ERR_ARG;
  g->ev_map = (int64_t*)calloc((size_t)x_bins * (size_t)rows, sizeof(int64_t));
  if (!g->ev_map) return ORC_ERR_ARG;
  g->ev_x = x_bins;
  g->ev_steps = steps_per_row;
  g->ev_rows = rows;
  return ORC_OK;
}

int orc_read_event_map(const orc_gap* g, int64_t* out) {
  if (!g || !g->ev_map || !out) return ORC_ERR_ARG;
  memcpy(out, g->ev_map, sizeof(int64_t) * (size_t)g->ev_x * (size_t)g->ev_rows);
  return ORC_OK;
}

static void record_history(orc_gap* g) {
  orc_history_row r;
  memset(&r, 0, sizeof r);
  r.step = g->step;
  r.n_minus = g->sp[0].n;
  r.n_plus = g->sp[1].n;
  r.n_photons = g->n_ph;
  r.pairs_created = g->pairs_created;
  r.photons_emitted = g->photons_emitted;
  r.photons_escaped = g->photons_escaped;
  r.absorbed_minus = g->absorbed[0];
  r.absorbed_plus = g->absorbed[1];
  double w = g->prm.weight;
  double ke = 0.0;
  for (int s = 0; s < 2; ++s)
    for (int64_t i = 0; i < g->sp[s].n; ++i) ke += w * gamma64(g->sp[s].p[i]);
  r.kinetic = ke;
  double fe = 0.0, es = 0.0;
  for (int32_t c = 0; c < g->prm.n_cells; ++c) {
    fe += g->E[c] * g->E[c] * g->prm.dx * 0.5;
    es += g->E[c];
  }
  r.field = fe;
  r.e_mean = es / (double)g->prm.n_cells;
  r.photon_energy = (double)g->n_ph * w * (g->prm.f * g->prm.gamma_thr);
  r.lost_energy = g->lost_energy;
  g->hist = (orc_history_row*)grow(g->hist, &g->cap_hist, g->n_hist + 1, sizeof(orc_history_row));
  g->hist[g->n_hist++] = r;
}

/* One step n: t^n -> t^{n+1}. */
static int step_once(orc_gap* g) {
  const orc_params* P = &g->prm;
  const int64_t ONE = g->one;
  const int64_t n = g->step;
  const double dtdx = R(g, P->dt / P->dx);
  const double scale = ldexp(1.0, g->K);
  const double gthr = R(g, P->gamma_thr);
  const double gpair = R(g, P->f * P->gamma_thr);
  const double ghalf = R(g, gpair * 0.5);
  const double pchild = R(g, sqrt(R(g, R(g, ghalf * ghalf) - 1.0)));
  const int64_t photon_step = (int64_t)rint(ldexp(P->dt / P->dx, g->K));
  const int64_t domain = (int64_t)P->n_cells * ONE;
  const int absorbing = P->boundary == ORC_BC_ABSORBING;

  int64_t n_pushed[2];
  int32_t* alive[2];
  double* gam_new[2];
  int nonfinite = 0;

  /* Ampere flux of this step starts from zero. */
  memset(g->F, 0, sizeof(int64_t) * (size_t)P->n_cells);

  /* 1-3. Gather, push, move and deposit, every lepton alive at t^n. */
  for (int s = 0; s < 2; ++s) {
    orc_species* S = &g->sp[s];
    const int64_t q = s == 0 ? -1 : 1;
    const double qdt = R(g, (double)q * P->dt);
    n_pushed[s] = S->n;
    alive[s] = (int32_t*)malloc(sizeof(int32_t) * (size_t)(S->n + 1));
    gam_new[s] = (double*)malloc(sizeof(double) * (size_t)(S->n + 1));
    for (int64_t i = 0; i < S->n; ++i) {
      int32_t c = S->cell[i];
      int64_t oq = S->offq[i];
      double o = ldexp((double)oq, -g->K);
      double Epart;
      int64_t jo = 0, Wo[3] = {0, 0, 0};
      if (P->shape == ORC_SHAPE_LINEAR) {
        /* gather: E averaged to the nodes c and c+1, then linear in the offset */
        double Em = R(g, e_ghost(g, c - 1)), Ec = R(g, e_ghost(g, c)), Ep = R(g, e_ghost(g, c + 1));
        double el = R(g, 0.5 * R(g, Em + Ec));
        double er = R(g, 0.5 * R(g, Ec + Ep));
        Epart = R(g, el + R(g, o * R(g, er - el)));
      } else {
        /* gather: E averaged to the nodes c+jo-1, c+jo, c+jo+1 (node k lies
         * between cells k-1 and k), weighted by the lepton's own spline
         * weights; jo is 0 or 1 */
        tsc_weights(g, oq, &jo, Wo);
        const int32_t k0 = c + (int32_t)jo - 1;
        double e[4];
        for (int k = 0; k < 4; ++k) e[k] = R(g, e_ghost(g, k0 - 1 + k));
        double en[3], sw[3];
        for (int k = 0; k < 3; ++k) {
          en[k] = R(g, 0.5 * R(g, e[k] + e[k + 1]));
          sw[k] = R(g, ldexp((double)Wo[k], -g->K));
        }
        Epart = R(g, R(g, R(g, sw[0] * en[0]) + R(g, sw[1] * en[1])) + R(g, sw[2] * en[2]));
      }
      /* push: p^{n+1/2} = p^{n-1/2} + q E dt */
      double p = R(g, S->p[i] + R(g, qdt * Epart));
      double gam = R(g, sqrt(R(g, 1.0 + R(g, p * p))));
      double v = R(g, p / gam);
      if (!isfinite(p) || !isfinite(gam)) nonfinite = 1;
      /* move: displacement in cells, rounded to the 2^-K grid */
      double d = R(g, v * dtdx);
      int64_t dq = (int64_t)rint(d * scale);
      int64_t nq = oq + dq;
      int keep = 1;
      if (P->shape == ORC_SHAPE_QUADRATIC) {
        /* charge-conserving deposit of the spline: the flux through cell k
         * (between nodes k and k+1) is the charge that left the nodes <= k,
         * the running sum of old minus new weight over nodes from the
         * leftmost one either spline touches; positions relative to node c.
         * A lepton leaving through an absorbing wall is carried on to 3/2
         * cells beyond it, where its spline no longer touches the wall node,
         * and removed; fluxes through cells outside the domain are dropped. */
        const int64_t X = (int64_t)c * ONE + nq;  /* from the left wall */
        int64_t target = nq;
        if (absorbing && X < 0) { target = -(ONE + ONE / 2) - (int64_t)c * ONE; keep = 0; }
        if (absorbing && X >= domain) {
          target = domain + ONE + ONE / 2 - (int64_t)c * ONE;
          keep = 0;
        }
        int64_t jn, Wn[3];
        tsc_weights(g, target, &jn, Wn);
        const int64_t lo = (jo < jn ? jo : jn) - 1, hi = (jo > jn ? jo : jn) + 1;
        int64_t run = 0;
        for (int64_t k = lo; k < hi; ++k) {
          const int64_t wo = (k >= jo - 1 && k <= jo + 1) ? Wo[k - jo + 1] : 0;
          const int64_t wn = (k >= jn - 1 && k <= jn + 1) ? Wn[k - jn + 1] : 0;
          run += wo - wn;
          const int64_t cell = (int64_t)c + k;
          if (absorbing) {
            if (cell >= 0 && cell < P->n_cells) g->F[cell] += q * run;
          } else {
            g->F[wrap_cell(g, (int32_t)cell)] += q * run;
          }
        }
        /* the lepton's own cell and offset after the move */
        if (keep) {
          if (nq >= ONE) { nq -= ONE; c = absorbing ? c + 1 : wrap_cell(g, c + 1); }
          else if (nq < 0) { nq += ONE; c = absorbing ? c - 1 : wrap_cell(g, c - 1); }
        }
      } else if (nq >= ONE) {
        g->F[c] += q * (ONE - oq);
        int32_t c1 = c + 1;
        nq -= ONE;
        if (c1 >= P->n_cells) {
          if (absorbing) keep = 0; else c1 = 0;
        }
        if (keep) g->F[c1] += q * nq;
        c = c1;
      } else if (nq < 0) {
        g->F[c] += q * (0 - oq);
        int32_t c1 = c - 1;
        nq += ONE;
        if (c1 < 0) {
          if (absorbing) keep = 0; else c1 = P->n_cells - 1;
        }
        if (keep) g->F[c1] += q * (nq - ONE);
        c = c1;
      } else {
        g->F[c] += q * dq;
      }
      S->p[i] = p;
      gam_new[s][i] = gam;
      alive[s][i] = keep;
      if (keep) {
        S->cell[i] = c;
        S->offq[i] = nq;
      } else {
        g->absorbed[s]++;
        g->lost_energy += P->weight * gamma64(p);
      }
    }
  }

  if (nonfinite) {
    for (int s = 0; s < 2; ++s) { free(alive[s]); free(gam_new[s]); }
    return ORC_ERR_NONFINITE;
  }

  /* 4. Ampere: E^{n+1} = E^n - J dt, with J dt = w * F * 2^-K; in the
   *    co-rotating frame (section 7) the imposed current adds j_m dt. */
  const double wq = ldexp(P->weight, -g->K);
  const double jmdt = P->j_m * P->dt;
  for (int32_t c = 0; c < P->n_cells; ++c) {
    double e = g->E[c] - wq * (double)g->F[c];
    if (jmdt != 0.0) e = e + jmdt;
    g->E[c] = e;
  }

  /* 5. Emission by the leptons that were pushed and survived. */
  int err = ORC_OK;
  for (int s = 0; s < 2 && err == ORC_OK; ++s) {
    orc_species* S = &g->sp[s];
    for (int64_t i = 0; i < n_pushed[s]; ++i) {
      if (!alive[s][i]) continue;
      double gm = gam_new[s][i];
      const double thr = P->gamma_thr_spread > 0.0 ? lepton_threshold(g, S->id[i]) : gthr;
      int k = 0;
      while (gm >= thr) {
        gm = R(g, gm - gpair);
        ++k;
        if (k > ORC_MAX_EMIT) { err = ORC_ERR_EMISSION; break; }
      }
      if (err != ORC_OK) break;
      if (k == 0) continue;
      double mag = R(g, sqrt(R(g, R(g, gm * gm) - 1.0)));
      int32_t dir = S->p[i] > 0.0 ? 1 : -1;
      S->p[i] = dir > 0 ? mag : -mag;
      int32_t c = S->cell[i];
      int64_t oq = S->offq[i];
      uint64_t id = S->id[i];
      for (int j = 0; j < k; ++j) {
        uint64_t bits;
        uint32_t u32;
        draw_run(id, P->seed, (uint64_t)n, (uint64_t)j, ORC_TAG_PHOTON, &bits, &u32);
        uint64_t child = bits & ~(uint64_t)1;
        g->photons_emitted++;
        if (g->table_len == 0) {
          /* in-place pair production (section 2) */
          append_pair(g, n, c, oq, dir, child, pchild);
          continue;
        }
        int64_t nc = conv_steps(g, u32);
        int64_t X = (int64_t)c * ONE + oq + (int64_t)dir * nc * photon_step;
        if (absorbing) {
          if (X < 0 || X >= domain) {
            g->photons_escaped++;
            g->lost_energy += P->weight * (P->f * P->gamma_thr);
            continue;
          }
        } else {
          X %= domain;
          if (X < 0) X += domain;
        }
        append_photon(g, X, n + nc, dir, child);
      }
    }
  }
  for (int s = 0; s < 2; ++s) free(gam_new[s]);
  if (err != ORC_OK) {
    for (int s = 0; s < 2; ++s) free(alive[s]);
    return err;
  }

  /* 6. Photons due at the end of this step become pairs. */
  int64_t kept = 0;
  for (int64_t i = 0; i < g->n_ph; ++i) {
    orc_photon ph = g->ph[i];
    if (ph.conv_step == n) {
      append_pair(g, n, (int32_t)(ph.xq / ONE), ph.xq % ONE, ph.dir, ph.child, pchild);
    } else {
      g->ph[kept++] = ph;
    }
  }
  g->n_ph = kept;

  /* Absorbed leptons leave the arrays (order is irrelevant to every result). */
  for (int s = 0; s < 2; ++s) {
    orc_species* S = &g->sp[s];
    int64_t w = 0;
    for (int64_t i = 0; i < S->n; ++i) {
      if (i < n_pushed[s] && !alive[s][i]) continue;
      S->cell[w] = S->cell[i]; S->offq[w] = S->offq[i]; S->p[w] = S->p[i]; S->id[w] = S->id[i];
      ++w;
    }
    S->n = w;
    free(alive[s]);
  }

  /* 7. Capacity: the step that overflows is not completed. */
  if (P->capacity > 0 && (g->sp[0].n > P->capacity || g->sp[1].n > P->capacity))
    return ORC_ERR_CAPACITY;

  /* 8. Diagnostics of the completed step. */
  record_history(g);
  g->step = n + 1;
  return ORC_OK;
}

int orc_step(orc_gap* g, int64_t n_steps) {
  if (!g || n_steps < 0) return ORC_ERR_ARG;
  if (g->status != ORC_OK) return ORC_ERR_STATE;
  for (int64_t i = 0; i < n_steps; ++i) {
    int st = step_once(g);
    if (st != ORC_OK) { g->status = st; return st; }
  }
  return ORC_OK;
}

int orc_status(const orc_gap* g) { return g->status; }
int64_t orc_steps_done(const orc_gap* g) { return g->step; }
int64_t orc_count(const orc_gap* g, int32_t species) {
  return (species == 0 || species == 1) ? g->sp[species].n : -1;
}
int64_t orc_photon_count(const orc_gap* g) { return g->n_ph; }

int orc_read_particles(const orc_gap* g, int32_t species, int64_t max_n, int32_t* cell,
                       double* off, double* p, uint64_t* id, int64_t* n_out) {
  if (!g || species < 0 || species > 1) return ORC_ERR_ARG;
  const orc_species* S = &g->sp[species];
  int64_t n = S->n < max_n ? S->n : max_n;
  for (int64_t i = 0; i < n; ++i) {
    if (cell) cell[i] = S->cell[i];
    if (off) off[i] = ldexp((double)S->offq[i], -g->K);
    if (p) p[i] = S->p[i];
    if (id) id[i] = S->id[i];
  }
  if (n_out) *n_out = S->n;
  return ORC_OK;
}

int orc_read_photons(const orc_gap* g, int64_t max_n, int64_t* xq, int64_t* conv_step,
                     int32_t* dir, uint64_t* child, int64_t* n_out) {
  if (!g) return ORC_ERR_ARG;
  int64_t n = g->n_ph < max_n ? g->n_ph : max_n;
  for (int64_t i = 0; i < n; ++i) {
    if (xq) xq[i] = g->ph[i].xq;
    if (conv_step) conv_step[i] = g->ph[i].conv_step;
    if (dir) dir[i] = g->ph[i].dir;
    if (child) child[i] = g->ph[i].child;
  }
  if (n_out) *n_out = g->n_ph;
  return ORC_OK;
}

/* rho: charge per node by the particle shape, integrated over a cell width
 * (Gauss: E_c - E_{c-1} = rho_c), nodes 0..n_cells (node n_cells is the
 * right wall; periodic folds it onto node 0). */
int orc_read_fields(const orc_gap* g, double* E, double* rho, int64_t* last_flux) {
  if (!g) return ORC_ERR_ARG;
  const int32_t N = g->prm.n_cells;
  if (E) memcpy(E, g->E, sizeof(double) * (size_t)N);
  if (last_flux) memcpy(last_flux, g->F, sizeof(int64_t) * (size_t)N);
  if (rho) {
    int64_t* acc = (int64_t*)calloc((size_t)N + 1, sizeof(int64_t));
    for (int s = 0; s < 2; ++s) {
      const int64_t q = s == 0 ? -1 : 1;
      for (int64_t i = 0; i < g->sp[s].n; ++i) {
        int32_t c = g->sp[s].cell[i];
        if (g->prm.shape == ORC_SHAPE_QUADRATIC) {
          int64_t j, W[3];
          tsc_weights(g, g->sp[s].offq[i], &j, W);
          for (int k = 0; k < 3; ++k) {
            int32_t node = c + (int32_t)j - 1 + k;
            if (g->prm.boundary == ORC_BC_PERIODIC) {   /* fold into [0, N) */
              node = node < 0 ? node + N : (node >= N ? node - N : node);
            } else if (node < 0 || node > N) {
              continue;                                  /* beyond a wall node */
            }
            acc[node] += q * W[k];
          }
          continue;
        }
        acc[c] += q * (g->one - g->sp[s].offq[i]);
        acc[c + 1] += q * g->sp[s].offq[i];
      }
    }
    if (g->prm.boundary == ORC_BC_PERIODIC) { acc[0] += acc[N]; acc[N] = acc[0]; }
    const double wq = ldexp(g->prm.weight, -g->K);
    for (int32_t c = 0; c <= N; ++c) rho[c] = wq * (double)acc[c];
    free(acc);
  }
  return ORC_OK;
}

int orc_set_fields(orc_gap* g, const double* E) {
  if (!g || !E) return ORC_ERR_ARG;
  for (int32_t c = 0; c < g->prm.n_cells; ++c) {
    if (!isfinite(E[c])) return ORC_ERR_ARG;
    g->E[c] = E[c];
  }
  return ORC_OK;
}

int orc_history(const orc_gap* g, orc_history_row* rows, int64_t max_rows, int64_t* n_out) {
  if (!g) return ORC_ERR_ARG;
  int64_t n = g->n_hist < max_rows ? g->n_hist : max_rows;
  if (rows && n > 0) memcpy(rows, g->hist, sizeof(orc_history_row) * (size_t)n);
  if (n_out) *n_out = g->n_hist;
  return ORC_OK;
}
