/* Drives the oracle (test infrastructure) through its API under the address
 * and undefined-behaviour sanitizers: built and run by
 * tests/test_oracle_sanitized.py with gcc -fsanitize=address,undefined.  Every
 * call's status is checked; any sanitizer report aborts the run. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pic_oracle.h"

#define CHECK(x)                                                          \
  do {                                                                    \
    if (!(x)) {                                                           \
      fprintf(stderr, "check failed: %s (line %d)\n", #x, __LINE__);      \
      exit(2);                                                            \
    }                                                                     \
  } while (0)

static orc_params base(void) {
  orc_params p;
  memset(&p, 0, sizeof p);
  p.n_cells = 128;
  p.dx = 1.0;
  p.dt = 0.45;
  p.boundary = ORC_BC_ABSORBING;
  p.e0 = 50.0;
  p.gamma_thr = 100.0;
  p.f = 0.5;
  p.l_gamma = 20.0;
  p.weight = 1.0;
  p.seed = 2012055870ull;
  p.precision = ORC_FP64;
  p.capacity = 0;
  return p;
}

/* Runs a gap for `steps` steps and reads back everything the API offers. */
static void run(orc_params p, int mode, int64_t pairs, int steps) {
  CHECK(orc_validate(&p) == ORC_OK);
  orc_gap* g = orc_create(&p);
  CHECK(g != NULL);
  CHECK(orc_event_map(g, 16, 10, 8) == ORC_OK);
  CHECK(orc_seed(g, mode, pairs, 4, 0.0, 0.0) == ORC_OK);
  CHECK(orc_seed(g, mode, pairs, 4, 0.0, 0.0) != ORC_OK); /* a second seeding is refused */
  const int st = orc_step(g, steps);
  CHECK(st == ORC_OK || st == ORC_ERR_CAPACITY);
  const int64_t done = orc_steps_done(g);
  CHECK(done >= 1 && done <= steps);
  for (int s = 0; s < 2; ++s) {
    const int64_t n = orc_count(g, s);
    CHECK(n >= 0);
    int32_t* cell = malloc(sizeof(int32_t) * (size_t)(n + 1));
    double* off = malloc(sizeof(double) * (size_t)(n + 1));
    double* mom = malloc(sizeof(double) * (size_t)(n + 1));
    uint64_t* id = malloc(sizeof(uint64_t) * (size_t)(n + 1));
    int64_t got = 0;
    CHECK(orc_read_particles(g, s, n, cell, off, mom, id, &got) == ORC_OK);
    CHECK(got == n);
    free(cell); free(off); free(mom); free(id);
  }
  const int64_t nph = orc_photon_count(g);
  int64_t* xq = malloc(sizeof(int64_t) * (size_t)(nph + 1));
  int64_t* cs = malloc(sizeof(int64_t) * (size_t)(nph + 1));
  int32_t* dir = malloc(sizeof(int32_t) * (size_t)(nph + 1));
  uint64_t* child = malloc(sizeof(uint64_t) * (size_t)(nph + 1));
  int64_t got = 0;
  CHECK(orc_read_photons(g, nph, xq, cs, dir, child, &got) == ORC_OK);
  CHECK(got == nph);
  free(xq); free(cs); free(dir); free(child);
  double* E = malloc(sizeof(double) * (size_t)p.n_cells);
  double* rho = malloc(sizeof(double) * (size_t)(p.n_cells + 1));
  int64_t* flux = malloc(sizeof(int64_t) * (size_t)p.n_cells);
  CHECK(orc_read_fields(g, E, rho, flux) == ORC_OK);
  orc_history_row* rows = malloc(sizeof(orc_history_row) * (size_t)(steps + 1));
  int64_t nrows = 0;
  CHECK(orc_history(g, rows, steps + 1, &nrows) == ORC_OK);
  CHECK(nrows == done);
  int64_t* map = malloc(sizeof(int64_t) * 16 * 8);
  CHECK(orc_read_event_map(g, map) == ORC_OK);
  free(map); free(rows); free(E); free(rho); free(flux);
  orc_destroy(g);
}

int main(void) {
  /* finite photon path with absorbing walls, both precisions and shapes */
  for (int prec = 0; prec < 2; ++prec)
    for (int shape = 0; shape < 2; ++shape) {
      orc_params p = base();
      p.precision = prec;
      p.shape = shape;
      run(p, ORC_SEED_RANDOM, 64, 120);
    }
  /* periodic, pairs in place, a spread of the threshold, lattice seed */
  {
    orc_params p = base();
    p.boundary = ORC_BC_PERIODIC;
    p.l_gamma = 0.0;
    p.gamma_thr_spread = 0.3;
    p.f = 0.1;
    run(p, ORC_SEED_LATTICE, 32, 80);
  }
  /* capacity freeze, imposed current, explicit seeding and set fields */
  {
    orc_params p = base();
    p.capacity = 600;
    p.j_m = 0.5;
    CHECK(orc_validate(&p) == ORC_OK);
    orc_gap* g = orc_create(&p);
    CHECK(g != NULL);
    double E[128];
    for (int c = 0; c < 128; ++c) E[c] = 50.0 * (1.0 - c / 256.0);
    CHECK(orc_set_fields(g, E) == ORC_OK);
    int32_t cell[3] = {3, 64, 127};
    double off[3] = {0.25, 0.5, 0.75}, mom[3] = {0.0, -1.0, 2.0};
    uint64_t id[3] = {10, 20, 30};
    CHECK(orc_seed_explicit(g, 0, 3, cell, off, mom, id) == ORC_OK);
    CHECK(orc_seed_explicit(g, 1, 3, cell, off, mom, id) == ORC_OK);
    const int st = orc_step(g, 400);
    CHECK(st == ORC_OK || st == ORC_ERR_CAPACITY);
    orc_destroy(g);
  }
  /* invalid parameters are rejected without touching memory */
  {
    orc_params p = base();
    p.n_cells = 1;
    CHECK(orc_validate(&p) != ORC_OK);
    CHECK(orc_create(&p) == NULL);
  }
  /* the generators and the table */
  {
    const uint64_t c64[4] = {1, 2, 3, 4}, k64[2] = {5, 6};
    uint64_t o64[4];
    orc_philox4x64_10(c64, k64, o64);
    const uint32_t c32[4] = {1, 2, 3, 4}, k32[2] = {5, 6};
    uint32_t o32[4];
    orc_philox4x32_10(c32, k32, o32);
    const int64_t n = orc_conv_table(0.45, 1.0, 20.0, NULL, 0);
    CHECK(n > 1);
    uint32_t* t = malloc(sizeof(uint32_t) * (size_t)n);
    CHECK(orc_conv_table(0.45, 1.0, 20.0, t, n) == n);
    CHECK(t[n - 1] == 0);
    free(t);
  }
  printf("oracle sanitized run: ok\n");
  return 0;
}
