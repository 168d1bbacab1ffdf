/*
 * pic.h -- C-ABI of the MI355X pair-cascade particle-in-cell library.
 *
 * The library advances one or many independent 1D "gaps": a line along the
 * magnetic field on which electrons and positrons are pushed by the parallel
 * field E, the field is advanced by Ampere's law, and leptons above a
 * threshold Lorentz factor emit pairs (Cruz, Grismayer & Silva, "Kinetic
 * model of large-amplitude oscillations in neutron star pair cascades",
 * arXiv:2012.05587).  The problem statement follows the paper: a uniform
 * initial field E0 over a domain of N cells, a seed pair plasma, the
 * threshold gamma_thr and the pair fraction f (sections 2 and 3); outputs are
 * the lepton counts N-(t) (Fig. 1), the momentum distributions and the E and
 * j profiles (Fig. 2), <E>(t) and n(t) (Fig. 3).
 *
 * Units are normalised: c = m_e = e = omega_p0 = 1.  x is in c/omega_p0,
 * t in 1/omega_p0, E in m_e c omega_p0 / e, momenta in m_e c, densities in
 * n0.  A macro-particle of weight w stands for a density w/dx.  Gauss's law
 * reads dE/dx = rho and Ampere's law (Eq. 4; Eq. 26 without the imposed
 * current) reads dE/dt = -J.
 *
 * Conventions shared by every call:
 *  - Every function returns a pic_status; PIC_OK is 0, errors are negative.
 *    No C++ exception crosses this boundary.
 *  - Memory.  The caller owns the device workspace (one allocation, any
 *    allocator, 256-byte aligned) and every host buffer.  The workspace must
 *    outlive the handle.  The library never allocates device memory and keeps
 *    no host pointer after a call returns.  Handles are host objects owned by
 *    the library and freed by pic_destroy / pic_destroy_batch.
 *  - Streams.  All device work is enqueued on the HIP stream given at
 *    creation (NULL = the null stream).  pic_step_n returns without waiting,
 *    except that with sort_every = 0 it keeps at most 8 of its timed graph
 *    replays in flight (a long call returns once all but the last 8 have
 *    run); pic_read_* and pic_set_fields synchronise that stream.
 *  - A handle is not thread-safe.
 *  - Capacity.  `capacity` bounds the live leptons of each species, as the
 *    model's memory bound: a step after which a species holds more live
 *    leptons than that is not completed.  The gap is frozen with
 *    PIC_ERR_CAPACITY; its step counter and history stay at the last
 *    completed step, while E and the particle arrays already hold that
 *    step's push and are not meaningful.  Later pic_step_n calls return
 *    PIC_ERR_STATE.  Each species has capacity + capacity/8 + 2048 slots:
 *    absorbed leptons keep their slots until the next re-sort, and a step
 *    whose appends do not fit the slots although the live leptons stay
 *    within capacity freezes the gap the same way with PIC_ERR_SLOTS.  The
 *    photon store has `photon_capacity` slots; converted and escaped photons
 *    keep theirs until the store is re-sorted, which a particle re-sort does
 *    once the store has gone unsorted for sqrt(128 m) steps (m the mean
 *    number of steps to conversion, at most 160) or is half full.  A step
 *    that overflows the store freezes with PIC_ERR_CAPACITY.
 *  - Non-finite momenta freeze the gap with PIC_ERR_NONFINITE the same way.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pic_status;
enum {
  PIC_OK = 0,
  PIC_ERR_ARG = -1,        /* invalid argument or parameter set */
  PIC_ERR_WORKSPACE = -2,  /* workspace too small or misaligned */
  PIC_ERR_CAPACITY = -3,   /* live leptons above the capacity, or photon store full */
  PIC_ERR_DEVICE = -4,     /* a HIP runtime call failed */
  PIC_ERR_STATE = -5,      /* wrong call order, or the gap is frozen */
  PIC_ERR_NONFINITE = -6,  /* a momentum became NaN or infinite */
  PIC_ERR_EMISSION = -7,   /* more than 64 emissions by one lepton in one step */
  PIC_ERR_SLOTS = -8       /* lepton slots exhausted by absorbed leptons not yet
                              reclaimed, while the live leptons fit the capacity */
};

enum { PIC_BC_PERIODIC = 0, PIC_BC_ABSORBING = 1 };
enum { PIC_FP64 = 0, PIC_MIXED = 1 };
enum { PIC_SEED_RANDOM = 0, PIC_SEED_LATTICE = 1 };
enum { PIC_SHAPE_LINEAR = 0, PIC_SHAPE_QUADRATIC = 1 };
enum { PIC_ELECTRON = 0, PIC_POSITRON = 1 };

/* Parameters of one gap.  Paper sections 2-3 give E0, gamma_thr, f, the
 * domain and the seed; the rest are numerical choices.
 *  n_cells   cells of width dx; E lives at cell centres, charge at nodes.
 *  dt        step; requires dt < dx (a lepton crosses at most one node).
 *  boundary  PIC_BC_PERIODIC or PIC_BC_ABSORBING (leptons leaving are
 *            removed after depositing their in-domain current; photons whose
 *            conversion point lies outside escape).
 *  e0        initial uniform field.
 *  gamma_thr a lepton with gamma >= gamma_thr emits (section 2).
 *  f         gamma_pair = f * gamma_thr is the energy of one emitted pair,
 *            split equally; requires 0 < f < 1, f*gamma_thr >= 2 and
 *            (1-f)*gamma_thr >= 1.  gamma_thr = +inf turns emission off.
 *  l_gamma   mean photon path in cells before conversion; 0 makes the pair
 *            in place, as in the paper's model.  Positions are int64
 *            multiples of 2^-K cells, so the domain and the longest photon
 *            path (about 22.2 l_gamma cells, where the conversion table ends)
 *            must each stay below 2^62 of them: with binary64 (K = 40) that
 *            is n_cells <= 2^22 and l_gamma below about 1.9e5 cells.
 *  weight    macro-particle weight w >= 0 (w = 0 gives test particles).
 *  capacity  live leptons per species at the end of a step (above it the
 *            gap freezes, see Capacity above); below 2^31 with its slot
 *            reserve.
 *  photon_capacity  slots of the photon store (l_gamma > 0); converted and
 *            escaped photons are reclaimed when the store is re-sorted.
 *  seed      key of this gap's random draws: the seeding draws are
 *            Philox4x64-10 blocks keyed by (pair index, seed); the draws of
 *            the run (photon paths and child ids, per-lepton thresholds) are
 *            Philox4x32-10 blocks at counter (step, j | tag << 8, id low 32
 *            bits, id high 32 bits), key (seed low, seed high), whose 64-bit
 *            value is word 1 << 32 | word 0 and whose 32-bit value is word 2.
 *  precision PIC_FP64: per-particle arithmetic in binary64, offsets on a
 *            2^-40 cell grid.  PIC_MIXED: binary32 push, offset (2^-24 grid)
 *            and momentum; the current, E and all diagnostics stay exact
 *            integer or binary64.
 *  sort_every   steps between particle re-sorts; 0 lets the library choose
 *               it while running (see pic_batch_tuning).  Between re-sorts,
 *               every 5 steps, the leptons appended since the last one are
 *               sorted among themselves in gaps wider than 2040 cells.  The
 *               cadence changes cost only: results do not depend on it while
 *               no gap runs out of slots (PIC_ERR_SLOTS).
 *  diag_every   steps between history rows (0 = 1).
 *  history_rows rows kept in the device history ring (0 = 4096).
 *  j_m       imposed current density of the frame co-rotating with the
 *            star (section 7): Ampere's law becomes dE/dt = -(J - j_m);
 *            0 everywhere else.
 *  gamma_thr_spread  sigma in [0, 1): a spread of the threshold, which the
 *            paper's conclusion names as absent from its model.  Each lepton
 *            then emits at its own fixed threshold, uniform in
 *            gamma_thr (1 - sigma, 1 + sigma): u = (top 53 bits of the 64-bit
 *            value of the lepton's draw at step 0, j 0, tag 3) / 2^53,
 *            threshold gamma_thr (1 + sigma (2u - 1)) in binary64,
 *            rounded to the particle precision.  gamma_pair stays
 *            f * gamma_thr.  Requires (1 - f - sigma) gamma_thr >= 1.  0 is
 *            the paper's single threshold.
 *  shape     particle shape, the same for every gap of a batch.
 *            PIC_SHAPE_LINEAR (0): cloud in cell, charge on the two nodes
 *            of the lepton's cell, node-averaged linear gather.
 *            PIC_SHAPE_QUADRATIC (1): quadratic spline over the nearest
 *            node j = floor(x + 1/2) and its neighbours, with d = x - j the
 *            fractions (1/2 - d)^2/2, 3/4 - d^2, (1/2 + d)^2/2 held as
 *            integers in 2^-K (outer two rounded down, the middle one the
 *            rest); the flux is the running sum of their change, so Gauss's
 *            law stays exact, and the gather weights node-averaged E with
 *            the same fractions.  At least 4 cells.  With absorbing walls
 *            the gather repeats the edge E (as for the linear shape), flux
 *            through cells beyond a wall is dropped, and a lepton leaving
 *            is carried 3/2 cells past the wall before it is removed, so
 *            that its charge leaves the wall node as current.             */
typedef struct {
  int32_t  n_cells;
  double   dx, dt;
  int32_t  boundary;
  double   e0;
  double   gamma_thr, f;
  double   l_gamma;
  double   weight;
  int64_t  capacity, photon_capacity;
  uint64_t seed;
  int32_t  precision;
  int32_t  sort_every, diag_every;
  int32_t  history_rows;
  double   j_m;
  double   gamma_thr_spread;
  int32_t  shape;
} pic_gap_params;

/* One row per diagnosed step (the quantities of Figs. 1 and 3). */
typedef struct {
  int64_t step;             /* index n of the completed step (state at t^{n+1}) */
  int64_t n_minus, n_plus;  /* live electrons / positrons */
  int64_t n_photons;        /* photons in flight */
  int64_t pairs_created;    /* cumulative */
  int64_t photons_emitted;  /* cumulative */
  int64_t photons_escaped;  /* cumulative */
  int64_t absorbed_minus, absorbed_plus; /* cumulative */
  double  kinetic;          /* sum w*gamma over live leptons, binary64 */
  double  field;            /* sum E_c^2 dx / 2 */
  double  photon_energy;    /* photons in flight times w*gamma_pair */
  double  lost_energy;      /* cumulative energy of absorbed leptons and escaped photons */
  double  e_mean;           /* <E> over the cells */
} pic_history_row;

typedef struct {
  int64_t steps_done;       /* completed steps */
  pic_status status;        /* PIC_OK or the error that froze the gap */
  int64_t pushes;           /* sum over completed steps of the leptons pushed */
} pic_step_report;

typedef struct {
  int64_t steps_done;
  pic_status status;
  int64_t n_minus, n_plus, n_photons;
  int64_t slots_minus, slots_plus, photon_slots; /* occupied slots (live + not yet reclaimed) */
  int64_t pushes;           /* cumulative leptons pushed */
  pic_history_row last;     /* the last history row written (zero before any step) */
  int64_t push_emissions;   /* cumulative photons (or in-place pairs) drawn by the push kernel
                               itself, in steps whose plan is small enough for it; the rest
                               are drawn by a later kernel of the step */
} pic_moments;

typedef struct pic_gap pic_gap;
typedef struct pic_batch pic_batch;

/* Checks a parameter set on the host.  PIC_OK or PIC_ERR_ARG. */
pic_status pic_validate_params(const pic_gap_params* p);

/* Device workspace, in bytes, needed by one gap with these parameters
 * (0 if the parameters are invalid). */
size_t pic_workspace_bytes(const pic_gap_params* p);

/* Creates a gap over caller-owned device memory d_ws of ws_bytes bytes on
 * HIP stream hip_stream (a hipStream_t, may be NULL).  E starts at e0 in
 * every cell; there are no particles.  *out receives the handle.
 * Errors: PIC_ERR_ARG (parameters, null out), PIC_ERR_WORKSPACE (size or
 * 256-byte alignment), PIC_ERR_DEVICE. */
pic_status pic_create_gap(const pic_gap_params* p, void* d_ws, size_t ws_bytes,
                          void* hip_stream, pic_gap** out);

/* Seeds n_pairs * macro_per_pair macro-pairs before the first step (the
 * uniform seed plasma of section 3).  Pair i holds an electron (id 2i) and a
 * positron (id 2i+1) at one point, so the seed is neutral.
 * PIC_SEED_RANDOM: u = Philox4x64-10(key (i, seed), counter (0, 0, 1, 0));
 * cell = (u0 >> 32) * n_cells >> 32, offset = (u1 >> 40) * 2^-24.
 * PIC_SEED_LATTICE: x_i = (i + 1/2) n_cells / N on the 2^-24 grid.
 * Momenta are p0_minus / p0_plus (taken as p at t = -dt/2).
 * The seed is sorted by cell group (8 cells) before the first step (by
 * pic_prepare or the first pic_step_n), so that its chunks deposit through
 * the LDS tile.
 * Errors: PIC_ERR_ARG, PIC_ERR_STATE (after the first step, or when the gap
 * already holds leptons: the seed ids start at 0), PIC_ERR_CAPACITY (more
 * pairs than the capacity), PIC_ERR_DEVICE. */
pic_status pic_seed_particles(pic_gap* g, int32_t mode, int64_t n_pairs,
                              int32_t macro_per_pair, double p0_minus, double p0_plus);

/* Appends n leptons of one species from host arrays (copied before return):
 * cell in [0, n_cells), offset in [0, 1) (rounded down to the offset grid),
 * momentum p, 64-bit id.  Only before the first step. */
pic_status pic_seed_explicit(pic_gap* g, int32_t species, int64_t n, const int32_t* cell,
                             const double* off, const double* p, const uint64_t* id);

/* Makes a seeded gap ready to step: enqueues the sort of the seed by cell
 * group and, on a non-NULL stream, captures and uploads the HIP graphs of the
 * step sequence (every candidate re-sort cadence when sort_every = 0), so
 * that pic_step_n only launches them.  Optional: pic_step_n does the same
 * work on first use.  Synchronises the stream.  Errors: PIC_ERR_STATE
 * after the first step, PIC_ERR_DEVICE. */
pic_status pic_prepare(pic_gap* g);

/* Enqueues n_steps steps.  Each step pushes every lepton in the field
 * gathered at its position, moves it with a charge-conserving current,
 * advances E by Ampere's law (Eq. 4), lets every lepton at or above
 * gamma_thr emit (section 2), converts the photons due at this step into
 * pairs and appends the new leptons.  Returns without waiting; *out (may be
 * NULL) is filled after a stream synchronisation if non-NULL.
 * Errors: PIC_ERR_STATE if the gap is already frozen; a new freeze is
 * reported by the status in *out, pic_read_moments, or the next call.
 * A gap runs at most 2^31 - 2^28 - 1 steps in all (photon conversion steps
 * are 32-bit); a call that would pass that enqueues nothing and returns
 * PIC_ERR_ARG. */
pic_status pic_step_n(pic_gap* g, int64_t n_steps, pic_step_report* out);

/* Copies E (n_cells binary64 values) and, if rho is non-NULL, the
 * cloud-in-cell node charge rho (n_cells + 1 values, integrated over a cell
 * so that E_c - E_{c-1} = rho_c) into host buffers.  Either may be NULL. */
pic_status pic_read_fields(pic_gap* g, double* E, double* rho, int32_t n_cells);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): pic_read_fields
 * computing rho in a static device array of (2^20 + 1) int64 node
 * accumulators, one per GPU, held from the first call on that GPU until the
 * process ends, instead of the workspace's.  Same arguments and results
 * (rho bit for bit), except that a gap of more than 2^20 cells gets
 * PIC_ERR_ARG when rho is requested.  Allocates no device or host memory:
 * the accumulators are copied into rho itself and converted in place.  The
 * array is cleared by a fill kernel at the start of each call; calls that
 * overlap on one GPU (several threads or streams) race on it and must be
 * serialised by the caller. */
pic_status pic_read_fields_noalloc(pic_gap* g, double* E, double* rho, int32_t n_cells);

/* Copies the flux sum q*w*(offset change) of the last step per cell, in
 * int64 units of w * 2^-K (K = 40 binary64, 24 mixed), into n_cells values. */
pic_status pic_read_flux(pic_gap* g, int64_t* flux, int32_t n_cells);

/* Counts, status and the last history row. */
pic_status pic_read_moments(pic_gap* g, pic_moments* out);

/* Copies up to max_rows history rows, oldest first (the ring keeps the
 * last history_rows rows); *n_out receives the number available. */
pic_status pic_read_history(pic_gap* g, pic_history_row* rows, int64_t max_rows,
                            int64_t* n_out);

/* Copies up to max_n live leptons of one species into host arrays (any of
 * them may be NULL); order is unspecified.  *n_out = live count. */
pic_status pic_read_particles(pic_gap* g, int32_t species, int64_t max_n, int32_t* cell,
                              double* off, double* p, uint64_t* id, int64_t* n_out);

/* Copies the photons in flight: conversion point in units of 2^-K cells,
 * conversion step, direction (+1/-1) and electron id of the future pair. */
pic_status pic_read_photons(pic_gap* g, int64_t max_n, int64_t* xq, int64_t* conv_step,
                            int32_t* dir, uint64_t* child, int64_t* n_out);

/* Overwrites E from a host buffer of n_cells finite values: a resume, or a
 * non-uniform initial field (the conclusion's field decaying with altitude).
 * The background charge dE/dx such a field implies is fixed and enters no
 * update (dE/dt depends on the current only). */
pic_status pic_set_fields(pic_gap* g, const double* E, int32_t n_cells);

/* Offset grid bits K of this gap (40 or 24). */
int32_t pic_offset_bits(const pic_gap* g);

/* ---- Diagnostics of the paper's figures, computed on the device. ----
 * Phase-space histogram of species s (0 electrons, 1 positrons) of gap g:
 * the momentum distributions of Fig. 2 (x_bins = 1) and the phase spaces
 * of section 7's figure.  A live lepton in cell c with momentum p counts in
 * d_counts[xb * p_bins + pb], xb = c * x_bins / n_cells (integer division),
 * pb = floor((p - p_min) * (p_bins / (p_max - p_min))) in binary64,
 * clamped to [0, p_bins).  d_counts is a caller-owned device array of
 * x_bins * p_bins int64 that the counts are added to; the work is enqueued
 * on the gap's stream (synchronise before reading).  Each count stands for
 * weight leptons.  Errors: PIC_ERR_ARG for a bad species, bin counts or
 * range. */
pic_status pic_phase_space(pic_gap* g, int32_t species, int32_t x_bins, int32_t p_bins,
                           double p_min, double p_max, int64_t* d_counts);
/* Pair-event map of section 7's figure (pair production events in x and
 * t).  From the next step on, every pair made at step n in cell c (in
 * place, or by a photon converting there) adds 1 to
 * d_map[row * x_bins + c * x_bins / n_cells], row = (n / steps_per_row) %
 * rows.  d_map is a caller-owned device array of rows * x_bins int64, kept
 * until the gap is destroyed or another call replaces it; the library
 * zeroes it on the gap's stream.  d_map = NULL stops the counting.
 * Synchronises the stream. */
pic_status pic_event_map(pic_gap* g, int64_t* d_map, int32_t x_bins, int32_t steps_per_row,
                         int32_t rows);

/* Frees the handle (not the workspace).  Synchronises the stream. */
pic_status pic_destroy(pic_gap* g);

const char* pic_status_string(pic_status s);

/* Kernel timing.  While enabled, every launch of the push kernel (gather,
 * push, move, current deposit and emission) carries HIP start and stop
 * events recorded by its dispatch on the gap's stream (steps are then
 * launched one by one, without graphs).  pic_read_push_time synchronises the stream and
 * returns the summed event time in milliseconds and the number of
 * launches timed since enabling; disabling clears the record. */
pic_status pic_profile_push(pic_gap* g, int32_t enable);
pic_status pic_read_push_time(pic_gap* g, double* ms, int64_t* launches);

/* ---- Batches: many independent gaps advanced by the same launches. ----
 * All gaps of a batch share precision, sort_every, diag_every and
 * history_rows (taken from params[0]); every other parameter is per gap.
 * The lepton capacities of a batch, both species, sum to less than 2^32.
 *
 * pic_batch_plan admits gaps in order while the total workspace stays
 * within budget_bytes: admitted[i] = 1 or 0; *ws_bytes = workspace of the
 * admitted set.  Returns the number admitted (>= 0) or PIC_ERR_ARG. */
int32_t    pic_batch_plan(const pic_gap_params* params, int32_t n_gaps, size_t budget_bytes,
                          uint8_t* admitted, size_t* ws_bytes);
size_t     pic_batch_workspace_bytes(const pic_gap_params* params, int32_t n_gaps);
pic_status pic_create_batch(const pic_gap_params* params, int32_t n_gaps, void* d_ws,
                            size_t ws_bytes, void* hip_stream, pic_batch** out);
/* Enqueues n_steps steps of every gap that is not frozen; per_gap (may be
 * NULL, n_gaps entries) receives each gap's status after a synchronisation.
 * The step limit of pic_step_n applies. */
pic_status pic_batch_step_n(pic_batch* b, int64_t n_steps, pic_status* per_gap);
/* Borrowed view of gap i, valid until pic_destroy_batch; usable with the
 * seed, read and set calls above (not with pic_step_n or pic_destroy). */
pic_gap*   pic_batch_gap(pic_batch* b, int32_t i);
int32_t    pic_batch_size(const pic_batch* b);
pic_status pic_destroy_batch(pic_batch* b);
/* Kernel timing of a batch, as pic_profile_push / pic_read_push_time. */
pic_status pic_batch_profile_push(pic_batch* b, int32_t enable);
pic_status pic_batch_read_push_time(pic_batch* b, double* ms, int64_t* launches);
/* pic_prepare for every gap of a batch. */
pic_status pic_batch_prepare(pic_batch* b);
/* Re-sort cadence.  The sort is not part of the paper's method: it only
 * reorders leptons for memory locality.  With sort_every = 0 the library times every
 * replayed graph of S steps plus the sort, S in {5, 10, 20, 40, 80}, and
 * every 16 replays probes half and twice the current S, switching when the
 * challenger is more than 2% faster per step.  Synchronises the stream.
 * Outputs (each may be NULL): the cadence in use, whether it is tuned, the
 * number of timed replays and of switches so far. */
pic_status pic_batch_tuning(pic_batch* b, int32_t* sort_every, int32_t* autotuned,
                            int64_t* replays, int32_t* switches);
/* The same for a single gap. */
pic_status pic_tuning(pic_gap* g, int32_t* sort_every, int32_t* autotuned, int64_t* replays,
                      int32_t* switches);

/* Where a step's emissions are drawn (section 2's emission: the photons, or
 * the pairs made in place, of the leptons that reached the threshold).  Not
 * part of the method: both kernels draw the same photons; only the cost
 * differs.  A step whose plan holds fewer than max_push_chunks lepton chunks
 * (1024 leptons of one species of one gap each) draws them inside the push
 * kernel, after each chunk; a larger step lists the emitters and a later
 * kernel of the step draws them, balanced by emitters.  Default 32768; 0
 * sends every step to the later kernel.  Applies to the whole batch from
 * the next step on.  Errors: PIC_ERR_ARG (null, max_push_chunks < 0),
 * PIC_ERR_DEVICE. */
pic_status pic_batch_emission_split(pic_batch* b, int64_t max_push_chunks);
pic_status pic_emission_split(pic_gap* g, int64_t max_push_chunks);

#ifdef __cplusplus
}
#endif
#endif
