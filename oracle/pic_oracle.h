/*
 * Oracle for the 1D pair-cascade particle-in-cell step -- TEST INFRASTRUCTURE.
 *
 * A plain, slow, scalar C implementation of what the data-parallel path
 * computes (Cruz, Grismayer & Silva, "Kinetic model of large-amplitude
 * oscillations in neutron star pair cascades", arXiv:2012.05587).  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or constant generator with the
 * HIP library; the two sides meet only through seeded inputs.
 *
 * Units are normalised: c = m_e = e = omega_p0 = 1; x in c/omega_p0, t in
 * 1/omega_p0, E in m c omega_p0 / e, densities in n0.  In these units Gauss's
 * law is dE/dx = rho and Ampere's law (Eq. 4 of section 3) is dE/dt = -J; in
 * the frame co-rotating with the star (section 7) they read
 * dE/dx = rho - rho_GJ and dE/dt = -(J - j_m), with the imposed current j_m.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_CAPACITY = -3, ORC_ERR_STATE = -5,
       ORC_ERR_NONFINITE = -6, ORC_ERR_EMISSION = -7 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_ABSORBING = 1 };
enum { ORC_FP64 = 0, ORC_MIXED = 1 };
enum { ORC_SEED_RANDOM = 0, ORC_SEED_LATTICE = 1 };
enum { ORC_SHAPE_LINEAR = 0, ORC_SHAPE_QUADRATIC = 1 };

typedef struct {
  int32_t  n_cells;
  double   dx, dt;
  int32_t  boundary;
  double   e0;          /* initial uniform field */
  double   gamma_thr;   /* emission threshold Lorentz factor */
  double   f;           /* gamma_pair = f * gamma_thr */
  double   l_gamma;     /* mean photon path in cells; 0 = pair made in place */
  double   weight;      /* macro-particle weight: density w/dx per macro */
  uint64_t seed;
  int32_t  precision;   /* ORC_FP64 or ORC_MIXED (per-particle arithmetic in binary32) */
  int64_t  capacity;    /* max live leptons per species; 0 = unlimited */
  double   j_m;         /* imposed current density (section 7, co-rotating frame):
                           dE/dt = -(J - j_m); 0 outside that setup */
  double   gamma_thr_spread; /* sigma in [0, 1): each lepton's threshold is fixed, uniform
                           in gamma_thr (1 - sigma, 1 + sigma), drawn from its id (the
                           spread the paper's conclusion names); 0 = one threshold */
  int32_t  shape;       /* particle shape: ORC_SHAPE_LINEAR (cloud in cell) or
                           ORC_SHAPE_QUADRATIC (quadratic spline over three nodes;
                           at least 4 cells) */
} orc_params;

typedef struct {
  int64_t step;            /* index n of the step just completed */
  int64_t n_minus, n_plus; /* live electrons / positrons after the step */
  int64_t n_photons;       /* photons in flight after the step */
  int64_t pairs_created;   /* cumulative pairs appended (in-place or converted) */
  int64_t photons_emitted; /* cumulative */
  int64_t photons_escaped; /* cumulative, absorbing boundary only */
  int64_t absorbed_minus, absorbed_plus; /* cumulative */
  double  kinetic;         /* sum w*gamma over live leptons (rest mass included), gamma
                              = sqrt(1 + p^2) in binary64 from the stored momentum */
  double  field;           /* sum E_c^2 dx / 2 */
  double  photon_energy;   /* energy carried by photons in flight */
  double  lost_energy;     /* cumulative energy of absorbed leptons and escaped photons */
  double  e_mean;          /* mean of E over the cells */
} orc_history_row;

typedef struct orc_gap orc_gap;

int      orc_validate(const orc_params* prm);
orc_gap* orc_create(const orc_params* prm);
void     orc_destroy(orc_gap* g);
int      orc_seed(orc_gap* g, int32_t mode, int64_t n_pairs, int32_t macro_per_pair,
                  double p0_minus, double p0_plus);
int      orc_seed_explicit(orc_gap* g, int32_t species, int64_t n, const int32_t* cell,
                           const double* off, const double* p, const uint64_t* id);
int      orc_step(orc_gap* g, int64_t n_steps);
int      orc_status(const orc_gap* g);
int64_t  orc_steps_done(const orc_gap* g);
int64_t  orc_count(const orc_gap* g, int32_t species);
int64_t  orc_photon_count(const orc_gap* g);
int      orc_read_particles(const orc_gap* g, int32_t species, int64_t max_n, int32_t* cell,
                            double* off, double* p, uint64_t* id, int64_t* n_out);
int      orc_read_photons(const orc_gap* g, int64_t max_n, int64_t* xq, int64_t* conv_step,
                          int32_t* dir, uint64_t* child, int64_t* n_out);
int      orc_read_fields(const orc_gap* g, double* E, double* rho, int64_t* last_flux);
int      orc_set_fields(orc_gap* g, const double* E);
int      orc_history(const orc_gap* g, orc_history_row* rows, int64_t max_rows, int64_t* n_out);
int      orc_offset_bits(const orc_gap* g);
/* Pair-event map: from now on every pair made at step n in cell c counts in
 * row (n / steps_per_row) % rows, column c * x_bins / n_cells (x_bins = 0
 * switches it off).  read copies rows x x_bins counts. */
int      orc_event_map(orc_gap* g, int32_t x_bins, int32_t steps_per_row, int32_t rows);
int      orc_read_event_map(const orc_gap* g, int64_t* out);

/* Building blocks exposed for pinning against libraries and closed forms. */
void     orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
void     orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int64_t  orc_conv_table(double dt, double dx, double l_gamma, uint32_t* table, int64_t max_len);

#ifdef __cplusplus
}
#endif
#endif
