"""Seeded synthetic workloads of the pair-cascade PIC path.

The paper (arXiv:2012.05587) runs its cascades on synthetic setups only: a
uniform seed pair plasma at rest in a uniform initial field (section 3), or
a co-rotating gap (section 7).  The workloads below keep that structure
(uniform seed, uniform E0, exponential cascade) at the sizes of the five
benchmark configurations.  This module only states parameters and draws
seeded gap tables; it holds none of the method's arithmetic, and both the
HIP path and the oracle take their inputs from it.

Enumerations follow the C-ABI: boundary 0 = periodic, 1 = absorbing;
precision 0 = binary64, 1 = mixed; seeding 0 = random, 1 = lattice.
"""
import math

import numpy as np

PERIODIC, ABSORBING = 0, 1
FP64, MIXED = 0, 1
SEED_RANDOM, SEED_LATTICE = 0, 1
BASE_SEED = 2012055870

# name -> gap parameters, seed plasma and run length
CONFIGS = {
    # 1: binary64 reference gap, small enough for the oracle in seconds
    "c1_fp64_reference_gap": dict(
        n_cells=512, dx=1.0, dt=0.45, boundary=ABSORBING, e0=50.0, gamma_thr=100.0, f=0.5,
        l_gamma=20.0, weight=1.0, seed=BASE_SEED + 1, precision=FP64, n_pairs=64,
        macro_per_pair=16, steps=2000, capacity=100_000, photon_capacity=100_000),
    # 2: binary64 single gap, cascade to ~1e7 macro-particles over 20000 steps
    "c2_fp64_single_gap": dict(
        n_cells=8192, dx=1.0, dt=0.45, boundary=ABSORBING, e0=200.0, gamma_thr=200.0, f=0.5,
        l_gamma=50.0, weight=1.0, seed=BASE_SEED + 2, precision=FP64, n_pairs=1024,
        macro_per_pair=1, steps=20000, capacity=30_000_000, photon_capacity=60_000_000),
    # 3: configuration 1 in mixed precision
    "c3_mixed_single_gap": dict(
        n_cells=512, dx=1.0, dt=0.45, boundary=ABSORBING, e0=50.0, gamma_thr=100.0, f=0.5,
        l_gamma=20.0, weight=1.0, seed=BASE_SEED + 1, precision=MIXED, n_pairs=64,
        macro_per_pair=16, steps=2000, capacity=100_000, photon_capacity=100_000),
    # 5: large mixed-precision gap, cascade to ~5e8 macro-particles
    "c5_large_mixed": dict(
        n_cells=65536, dx=1.0, dt=0.45, boundary=ABSORBING, e0=1000.0, gamma_thr=500.0, f=0.5,
        l_gamma=200.0, weight=1.0, seed=BASE_SEED + 5, precision=MIXED, n_pairs=16384,
        macro_per_pair=1, steps=50000, capacity=300_000_000, photon_capacity=300_000_000,
        sort_every=20),
}

GAP_KEYS = ("n_cells", "dx", "dt", "boundary", "e0", "gamma_thr", "f", "l_gamma", "weight",
            "seed", "precision")


def config(name):
    return dict(CONFIGS[name])


def batched_scan(n_gaps=256, precision=MIXED, steps=2000, seed=BASE_SEED):
    """Configuration 4: independent gaps with log-uniform N_cells in
    [1024, 16384], E0 and gamma_thr uniform in [50, 400], l_gamma uniform in
    [10, 100] cells and log-uniform 256-4096 seed pairs; f = 0.5, dt = 0.45,
    dx = 1, absorbing.  Slots per species are sized from the seed-to-screening
    growth bound 3 * 2 * (E0^2 ln(2/f) / (2 gamma_thr)) * N_cells, clipped to
    [1e5, 1e7]."""
    rng = np.random.default_rng(seed)
    gaps = []
    for i in range(n_gaps):
        nc = int(round(math.exp(rng.uniform(math.log(1024), math.log(16384)))))
        e0 = float(rng.uniform(50.0, 400.0))
        gthr = float(rng.uniform(50.0, 400.0))
        lg = float(rng.uniform(10.0, 100.0))
        pairs = int(round(math.exp(rng.uniform(math.log(256), math.log(4096)))))
        ns = e0 * e0 * math.log(2.0 / 0.5) / (2.0 * gthr)
        cap = int(min(max(3 * 2 * ns * nc, 1e5), 1e7))
        gaps.append(dict(n_cells=nc, dx=1.0, dt=0.45, boundary=ABSORBING, e0=e0, gamma_thr=gthr,
                         f=0.5, l_gamma=lg, weight=1.0, seed=seed + 1000 + i,
                         precision=precision, n_pairs=pairs, macro_per_pair=1, steps=steps,
                         capacity=cap, photon_capacity=cap))
    return gaps


def corotating_gap(n_cells=10000, dx=0.1, dt=1e-3, ppc_plus=10, gamma_thr=5000.0, f=0.01,
                   l_gamma=0.0, precision=MIXED, steps=20000, capacity=20_000_000,
                   photon_capacity=0, seed=BASE_SEED + 7):
    """The co-rotating polar-cap gap of section 7: Goldreich-Julian density
    n_GJ = |rho_GJ| / e is the density unit (rho_GJ = -1), the magnetosphere
    imposes j_m = -1.5 rho_GJ c = 1.5, and the walls are open (leptons that
    leave are removed).  Positrons at density 1 and electrons at density 2,
    evenly spaced, make rho = rho_GJ with E = 0; cold velocities -0.5 c
    (electrons) and +0.5 c (positrons), i.e. momenta -/+1/sqrt(3), make
    J = 2 * 0.5 + 1 * 0.5 = j_m.  Defaults: the paper's L = 1000, dx = 0.1,
    dt = 1e-3 (in units of c / omega_p,GJ and 1 / omega_p,GJ), gamma_thr =
    5000 and f = 0.01 with pairs made in place.

    Returns the gap configuration with the explicit seed in "explicit":
    species -> (cell, offset, momentum, id), offsets on the 2^-24 grid."""
    n_plus = ppc_plus * n_cells
    n_minus = 2 * n_plus
    weight = dx / ppc_plus  # one macro-positron per cell at density 1 gives w / dx
    p_cold = 1.0 / math.sqrt(3.0)
    explicit = {}
    for sp, n, p0 in ((0, n_minus, -p_cold), (1, n_plus, p_cold)):
        i = np.arange(n, dtype=np.int64)
        X = ((2 * i + 1) * n_cells * (1 << 24)) // (2 * n)  # (i + 1/2) L / n on the 2^-24 grid
        cell = (X >> 24).astype(np.int32)
        off = (X & 0xFFFFFF).astype(np.float64) / float(1 << 24)
        p = np.full(n, p0)
        ids = 2 * i.astype(np.uint64) + np.uint64(sp)
        explicit[sp] = (cell, off, p, ids)
    return dict(n_cells=n_cells, dx=dx, dt=dt, boundary=ABSORBING, e0=0.0, gamma_thr=gamma_thr,
                f=f, l_gamma=l_gamma, weight=weight, seed=seed, precision=precision, n_pairs=0,
                macro_per_pair=1, steps=steps, capacity=capacity,
                photon_capacity=photon_capacity, j_m=1.5, rho_gj=-1.0, explicit=explicit)


def uniform_cascade(f, gamma_thr=500.0, n_cells=2000, precision=MIXED, seed=BASE_SEED + 30,
                    gamma_thr_spread=0.0, steps=12000, shape=0):
    """The cascade of sections 3-5 at the resolution of the paper's runs: a
    uniform seed of pairs at rest (one pair per cell, random positions) in
    a uniform field E0 = 10^3.5, periodic, pairs made in place, gamma_thr =
    500 (larger where f * gamma_thr < 2 would leave the pair below two rest
    masses), L = 10^1.5 c/omega_p0 over n_cells cells, dt = 10^-3.5 and
    macro-particle weight dx (seed density 1 per species).  Slots per
    species: 1.25 * E0^2 ln(2/f) / (2 gamma_thr) * n_cells.  gamma_thr_spread
    gives each lepton its own threshold, uniform in gamma_thr (1 +/- spread);
    shape 1 the quadratic-spline particle shape."""
    L = 10.0 ** 1.5
    dx = L / n_cells
    e0, gthr = 10.0 ** 3.5, float(gamma_thr)
    cap = int(1.25 * e0 * e0 * math.log(2.0 / f) / (2.0 * gthr) * n_cells)
    return dict(n_cells=n_cells, dx=dx, dt=10.0 ** -3.5, boundary=PERIODIC, e0=e0,
                gamma_thr=gthr, f=f, l_gamma=0.0, weight=dx, seed=seed, precision=precision,
                n_pairs=n_cells, macro_per_pair=1, seed_mode=SEED_RANDOM, capacity=cap,
                photon_capacity=0, gamma_thr_spread=gamma_thr_spread, steps=steps, shape=shape)


def nonuniform_gap(n_cells=2000, length=10.0 ** 1.5, dt=10.0 ** -3.5, e0=10.0 ** 3.5,
                   e_scale=0.25, seed_pairs=2000, seed_scale=0.25, gamma_thr=500.0, f=0.1,
                   l_gamma=0.0, weight=None, precision=MIXED, steps=20000, capacity=None,
                   photon_capacity=0, seed=BASE_SEED + 40):
    """A gap with the non-uniform start that the paper's conclusion names as
    a limitation of its uniform runs: the field decays with altitude and so
    does the seed.  The surface is the left wall (x = 0), walls absorbing.
    Defaults: the resolution and E0 of the section 3 runs (2000 cells over
    L = 10^1.5, dt = 10^-3.5, surface field 10^3.5, gamma_thr = 500), f = 0.1,
    pairs made in place, weight dx (mean seed density 1 per species).

    E(x) = e0 exp(-x / (e_scale L)) at the cell centres x = (c + 1/2) dx,
    in "E_init"; Gauss's law then holds with a fixed background charge
    dE/dx.  Seed pairs at rest, electron and positron at the same point, at
    positions drawn from the density exp(-x / (seed_scale L)) on [0, L)
    (inverse CDF of numpy's default_rng uniforms), on the 2^-24 grid.
    Slots per species by default: 1.25 E0^2 ln(2/f) / (2 gamma_thr) L / w,
    the uniform gap's bound.  Returns the configuration with the explicit
    seed in "explicit"."""
    L = float(length)
    dx = L / n_cells
    w = dx if weight is None else float(weight)
    if capacity is None:
        capacity = int(1.25 * e0 * e0 * math.log(2.0 / f) / (2.0 * gamma_thr) * L / w)
    xc = (np.arange(n_cells) + 0.5) * dx
    E = e0 * np.exp(-xc / (e_scale * L))
    rng = np.random.default_rng(seed)
    u = rng.random(seed_pairs)
    ls = seed_scale * L
    x = -ls * np.log1p(-u * -np.expm1(-L / ls))
    X = np.minimum(np.floor(x / dx * (1 << 24)).astype(np.int64), n_cells * (1 << 24) - 1)
    cell = (X >> 24).astype(np.int32)
    off = (X & 0xFFFFFF).astype(np.float64) / float(1 << 24)
    i = np.arange(seed_pairs, dtype=np.uint64)
    explicit = {sp: (cell, off, np.zeros(seed_pairs), 2 * i + np.uint64(sp)) for sp in (0, 1)}
    return dict(n_cells=n_cells, dx=dx, dt=dt, boundary=ABSORBING, e0=e0, gamma_thr=gamma_thr,
                f=f, l_gamma=l_gamma, weight=w, seed=seed, precision=precision, n_pairs=0,
                macro_per_pair=1, steps=steps, capacity=capacity,
                photon_capacity=photon_capacity, E_init=E, explicit=explicit)


def stream_lattice(n_pairs=100_000_000, n_cells=65536, precision=MIXED, steps=200,
                   seed=BASE_SEED + 50):
    """The push alone: emission off (gamma_thr = inf), periodic, n_pairs
    pairs on the lattice x_i = (i + 1/2) n_cells / N at rest, E0 = 1, weight
    1e-6 (so the plasma barely moves the field).  Every chunk stays sorted
    and nothing is appended, so the step is one streaming push of every
    lepton plus the cheap field update."""
    return dict(n_cells=n_cells, dx=1.0, dt=0.45, boundary=PERIODIC, e0=1.0,
                gamma_thr=float("inf"), f=0.5, l_gamma=0.0, weight=1e-6, seed=seed,
                precision=precision, n_pairs=n_pairs, macro_per_pair=1,
                seed_mode=SEED_LATTICE, steps=steps, capacity=n_pairs, photon_capacity=0)


def scaled(name, **over):
    """A configuration with some fields replaced (smaller parity cases)."""
    c = config(name)
    c.update(over)
    return c
