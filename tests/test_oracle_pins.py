"""Pins of the oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  Each checks the oracle against something
other than itself: a library routine (numpy's Philox), a closed form (test
particle, leapfrog cold-plasma dispersion), an invariant (Gauss's law, pair
bookkeeping), brute force on a tiny case, or the paper's analytic results
(growth rate of section 3, screening density of Eq. 5, energy balance of
section 4 and Eq. 10, oscillation frequency of section 5).
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle
from oracle import analytic as A
from tests import brute_tree


def _np_philox(ctr, key):
    return np.array(brute_tree.philox(ctr, key), dtype=np.uint64)


# --------------------------------------------------------------------------- RNG
@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (0, 0)),
    ((7, 3, 2, 0), (12345, 2012055870)),
    ((2**64 - 1, 2**64 - 1, 5, 0), (2**63 + 5, 77)),
    ((123456789, 63, 2, 0), (0xFFFFFFFFFFFFFFFE, 2012055875)),
])
def test_philox_matches_numpy(ctr, key):
    """Philox4x64-10 (SC'11) bit for bit against numpy.random.Philox."""
    assert (oracle.philox4x64_10(ctr, key) == _np_philox(ctr, key)).all()


# Published known-answer vectors of Philox4x32-10 (Salmon et al., SC'11; the
# Random123 distribution's tests): counter, key -> output words.
PHILOX4X32_KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,want", PHILOX4X32_KAT)
def test_philox4x32_known_answers(ctr, key, want):
    """Philox4x32-10, which draws each emission's child id and photon path and
    each lepton's threshold, reproduces the generator's published
    known-answer vectors, in the oracle and in the brute-force helper."""
    assert [int(x) for x in oracle.philox4x32_10(ctr, key)] == list(want)
    assert brute_tree.philox4x32(ctr, key) == list(want)


def test_philox4x32_oracle_matches_helper_on_run_counters():
    """The oracle's block and the helper's agree on counters of the run's
    layout (step, j | tag << 8, id low, id high) and 64-bit seeds."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        pid = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        seed = int(rng.integers(0, 2**63))
        step, j, tag = int(rng.integers(0, 2**31)), int(rng.integers(0, 65)), int(rng.integers(2, 4))
        ctr = (step, j | (tag << 8), pid & 0xFFFFFFFF, pid >> 32)
        key = (seed & 0xFFFFFFFF, seed >> 32)
        assert [int(x) for x in oracle.philox4x32_10(ctr, key)] == brute_tree.philox4x32(ctr, key)


# ----------------------------------------------------------------- photon path
def test_conversion_table_is_floor_of_geometric_tail():
    """T_k = floor(q^k 2^32), q = exp(-dt/(l_gamma dx)), checked with 40-digit
    decimal arithmetic instead of libm."""
    dt, dx, lg = 0.45, 1.0, 20.0
    t = oracle.conv_table(dt, dx, lg)
    getcontext().prec = 40
    r = Decimal(dt) / (Decimal(lg) * Decimal(dx))
    assert t[-1] == 0 and t[-2] > 0
    mismatches = 0
    for k in range(len(t)):
        exact = (-(Decimal(k) * r)).exp() * (Decimal(2) ** 32)
        fl = int(exact)  # floor for positive values
        if k == 0:
            assert t[0] == 0xFFFFFFFF
            continue
        if t[k] != min(fl, 0xFFFFFFFF):
            # libm rounding may only matter within a hair of an integer
            assert abs(exact - Decimal(t[k] + 1)) < Decimal("1e-6") or \
                abs(exact - Decimal(t[k])) < Decimal("1e-6")
            mismatches += 1
    assert mismatches <= 1
    # length: q^k 2^32 < 1  <=>  k > 32 ln2 / r
    assert abs(len(t) - 1 - math.ceil(32 * math.log(2) / (dt / lg))) <= 1


def test_conversion_steps_follow_discretised_exponential():
    """n_conv = min{k>=1 : u >= T_k} has P(n_conv > k) = q^k: its mean is
    1/(1-q), i.e. ceil(S/(c dt)) for an exponential path S of mean l_gamma."""
    dt, dx, lg = 0.45, 1.0, 20.0
    t = oracle.conv_table(dt, dx, lg).astype(np.int64)
    rng = np.random.default_rng(5)
    u = rng.integers(0, 2**32, size=200_000, dtype=np.int64)
    # first k >= 1 with u >= T_k; T is decreasing so use searchsorted on -T
    k = np.searchsorted(-t[1:], -u, side="left") + 1
    q = math.exp(-dt / (lg * dx))
    mean = 1.0 / (1.0 - q)
    sd = math.sqrt(q) / (1.0 - q)
    assert abs(k.mean() - mean) < 5 * sd / math.sqrt(len(u))
    for kk in (1, 10, 50, 200):
        emp = (k > kk).mean()
        assert abs(emp - q**kk) < 5 * math.sqrt(q**kk * (1 - q**kk) / len(u)) + 1e-9


# ------------------------------------------------------------- test particle
def _test_particle(e0, dt, n_steps, p0=0.0, species=1, precision=oracle.FP64):
    g = oracle.OracleGap(n_cells=64, dx=1.0, dt=dt, boundary=oracle.PERIODIC, e0=e0,
                         gamma_thr=1e300, f=0.5, l_gamma=0.0, weight=0.0, seed=1,
                         precision=precision)
    g.seed_explicit(species, [3], [0.25], [p0], [9])
    ps, xs = [], []
    for _ in range(n_steps):
        assert g.step(1) == oracle.OK
        P = g.particles(species)
        ps.append(P["p"][0])
        xs.append(P["cell"][0] + P["off"][0])
    return np.array(ps), np.array(xs)


def test_test_particle_momentum_closed_form():
    """Weight 0 (no current) in a uniform field: p^{n+1/2} = p0 + (n+1) q E0 dt,
    to within one rounding per step."""
    e0, dt, p0 = 3.0, 0.3, -2.5
    for species, q in ((0, -1.0), (1, 1.0)):
        ps, _ = _test_particle(e0, dt, 400, p0=p0, species=species)
        n = np.arange(400)
        exact = p0 + (n + 1) * q * e0 * dt
        ulp = np.spacing(np.abs(exact) + 1.0)
        assert np.all(np.abs(ps - exact) <= (n + 2) * ulp)


def test_test_particle_position_second_order():
    """x(t) = x0 + (gamma(t) - gamma(t0)) / (q E0) for hyperbolic motion; the
    leapfrog error at fixed time falls by ~4 when dt is halved."""
    e0 = 0.5
    T = 12.0
    errs = []
    for dt in (0.2, 0.1, 0.05):
        n = int(round(T / dt))
        ps, xs = _test_particle(e0, dt, n, p0=0.0, species=1)
        # exact: p(t) = E0 (t + dt/2) from p(-dt/2) = 0; position at t = n dt
        t_end = n * dt
        p_exact0 = e0 * dt / 2
        g0 = math.sqrt(1 + p_exact0**2)
        g1 = math.sqrt(1 + (e0 * (t_end + dt / 2)) ** 2)
        # the particle drifts across the periodic box: unwrap by cell count
        x_exact = 3.25 + (g1 - g0) / e0
        x_num = xs[-1]
        wraps = round((x_exact - x_num) / 64.0)
        errs.append(abs(x_num + 64.0 * wraps - x_exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, errs


# ------------------------------------------------------------------- Gauss
@pytest.mark.parametrize("boundary", [oracle.ABSORBING, oracle.PERIODIC])
@pytest.mark.parametrize("precision", [oracle.FP64, oracle.MIXED])
def test_gauss_residual_at_roundoff(boundary, precision):
    """The charge-conserving deposit keeps E_c - E_{c-1} = rho_c at every
    (interior) node, to round-off accumulated by the field update."""
    g = oracle.OracleGap(n_cells=128, dx=1.0, dt=0.45, boundary=boundary, e0=20.0,
                         gamma_thr=60.0, f=0.5, l_gamma=8.0, weight=0.5, seed=11,
                         precision=precision)
    g.seed(oracle.SEED_RANDOM, 256, 1)
    steps = 300
    assert g.step(steps) == oracle.OK
    F = g.fields()
    E, rho = F["E"], F["rho"]
    if boundary == oracle.PERIODIC:
        r = (E - np.roll(E, 1)) - rho[:-1]
    else:
        r = (E[1:] - E[:-1]) - rho[1:-1]
    bound = 10 * np.finfo(float).eps * steps * np.abs(E).max()
    assert np.abs(r).max() <= bound
    assert g.history()["pairs_created"][-1] > 256  # the cascade did run


# ----------------------------------------------------------- uniform drift
@pytest.mark.parametrize("shape", [oracle.SHAPE_LINEAR, oracle.SHAPE_QUADRATIC])
@pytest.mark.parametrize("precision", [oracle.FP64, oracle.MIXED])
def test_uniform_lattice_drift_flux_is_uniform_and_exact(shape, precision):
    """A lattice of one species drifting at one velocity in zero field puts the
    same integer flux m * dq through every cell (m macros per cell), for
    either particle shape."""
    m, nc = 4, 32
    dt, dx, p = 0.45, 1.0, 3.7
    g = oracle.OracleGap(n_cells=nc, dx=dx, dt=dt, boundary=oracle.PERIODIC, e0=0.0,
                         gamma_thr=1e300, f=0.5, l_gamma=0.0, weight=0.0, seed=1,
                         shape=shape, precision=precision)
    N = m * nc
    x = np.floor((np.arange(N) + 0.5) * (nc / N) * 2**24).astype(np.int64)
    g.seed_explicit(0, x >> 24, (x & 0xFFFFFF) / 2**24, np.full(N, p), np.arange(N) * 2)
    K = g.offset_bits
    for _ in range(5):
        assert g.step(1) == oracle.OK
        flux = g.fields()["flux"]
        pr = p if precision == oracle.FP64 else float(np.float32(p))
        if precision == oracle.FP64:
            v = pr / math.sqrt(1 + pr * pr)
            dq = round(v * (dt / dx) * 2**K)
        else:
            f32 = np.float32
            gam = f32(np.sqrt(f32(f32(1) + f32(pr) * f32(pr))))
            v = f32(f32(pr) / gam)
            dq = int(np.rint(f32(v * f32(dt / dx)) * f32(2**K)))
        assert np.all(flux == -m * dq)


# ------------------------------------------------------------- cold plasma
@pytest.mark.parametrize("shape", [oracle.SHAPE_LINEAR, oracle.SHAPE_QUADRATIC])
def test_cold_plasma_frequency_matches_leapfrog_dispersion(shape):
    """Uniform co-located pairs (n per species) in a small uniform field
    oscillate at sin(omega dt/2) = omega_p dt/2, omega_p^2 = 2n (the uniform
    mode does not see the particle shape)."""
    from scipy.optimize import curve_fit
    nc, dx, dt, e0 = 8, 1.0, 0.45, 1e-3
    g = oracle.OracleGap(n_cells=nc, dx=dx, dt=dt, boundary=oracle.PERIODIC, e0=e0,
                         gamma_thr=1e300, f=0.5, l_gamma=0.0, weight=1.0, seed=1, shape=shape)
    g.seed(oracle.SEED_LATTICE, nc, 1)
    n_per_species = 1.0 * 1 / dx
    omega = A.leapfrog_cold_frequency(n_per_species, dt)
    periods = 24
    steps = int(periods * 2 * math.pi / omega / dt)
    assert g.step(steps) == oracle.OK
    Em = g.history()["e_mean"]
    t = np.arange(1, steps + 1) * dt

    def model(t, a, w, ph, b):
        return a * np.cos(w * t + ph) + b

    p0 = (e0, omega * (1 + 1e-4), 0.0, 0.0)
    # initial phase from the first sample
    popt, _ = curve_fit(model, t, Em, p0=p0, maxfev=20000)
    assert abs(popt[1] / omega - 1.0) < 1e-6
    # and the continuum frequency sqrt(2n) is measurably different
    assert abs(popt[1] / math.sqrt(2 * n_per_species) - 1.0) > 1e-2


# ------------------------------------------------------------ brute force
@pytest.mark.parametrize("l_gamma,absorbing,spread,shape", [
    (0.0, True, 0.0, 0), (6.0, True, 0.0, 0), (6.0, False, 0.0, 0), (0.0, True, 0.3, 0),
    (6.0, False, 0.3, 0), (6.0, False, 0.0, 1), (6.0, True, 0.0, 1)])
def test_frozen_field_tree_matches_brute_force(l_gamma, absorbing, spread, shape):
    """Zero weight freezes E at E0; per-step lepton, photon, conversion, escape
    and absorption counts and every final lepton agree exactly with an
    independent lineage-by-lineage simulation using numpy's Philox (also with
    a spread of the threshold, each lepton's own drawn there independently)."""
    prm = dict(n_cells=48, dx=1.0, dt=0.45,
               boundary=oracle.ABSORBING if absorbing else oracle.PERIODIC,
               e0=50.0, gamma_thr=100.0, f=0.5, l_gamma=l_gamma, weight=0.0, seed=2012055870,
               gamma_thr_spread=spread, shape=shape)
    steps = 32 if l_gamma == 0.0 else 60
    g = oracle.OracleGap(**prm)
    g.seed(oracle.SEED_RANDOM, 3, 1)
    seeds = []
    for s in (0, 1):
        P = g.particles(s)
        for c, o, p, i in zip(P["cell"], P["off"], P["p"], P["id"]):
            seeds.append((s, int(c), int(round(o * 2**40)), float(p), int(i)))
    assert g.step(steps) == oracle.OK
    ref = brute_tree.run(prm["n_cells"], prm["dx"], prm["dt"], absorbing, prm["e0"],
                         prm["gamma_thr"], prm["f"], l_gamma, seeds, steps, prm["seed"],
                         gamma_thr_spread=spread)
    h = g.history()
    for key in ("n_minus", "n_plus", "n_photons", "photons_emitted", "photons_escaped",
                "pairs_created", "absorbed_minus", "absorbed_plus"):
        assert np.array_equal(h[key], ref[key]), key
    final = {}
    for s in (0, 1):
        P = g.particles(s)
        for c, o, p, i in zip(P["cell"], P["off"], P["p"], P["id"]):
            final[int(i)] = (s, int(c), int(round(o * 2**40)), float(p))
    assert final == ref["final"]
    assert h["pairs_created"][-1] > 20


# ------------------------------------------------------------ bookkeeping
def test_pair_and_photon_bookkeeping_invariants():
    """N- - N+ changes only by absorption; every emitted photon is in flight,
    converted or escaped; lost energy only grows."""
    g = oracle.OracleGap(n_cells=512, dx=1.0, dt=0.45, boundary=oracle.ABSORBING, e0=50.0,
                         gamma_thr=100.0, f=0.5, l_gamma=20.0, weight=1.0, seed=2012055870)
    g.seed(oracle.SEED_RANDOM, 64, 16)
    assert g.step(400) == oracle.OK
    h = g.history()
    assert np.all((h["n_minus"] - h["n_plus"]) == -(h["absorbed_minus"] - h["absorbed_plus"]))
    assert np.all(h["photons_emitted"] == h["n_photons"] + h["pairs_created"] + h["photons_escaped"])
    assert np.all(np.diff(h["lost_energy"]) >= 0)
    assert np.all(np.diff(h["pairs_created"]) >= 0)


def test_emission_conserves_energy_in_frozen_field():
    """In a frozen field the only energy source is the work q E0 v dt; emission
    itself moves gamma_pair from the emitter to the pair exactly (in-place)."""
    e0, dt = 50.0, 0.45
    g = oracle.OracleGap(n_cells=4096, dx=1.0, dt=dt, boundary=oracle.PERIODIC, e0=e0,
                         gamma_thr=100.0, f=0.5, l_gamma=0.0, weight=1e-300, seed=3)
    g.seed(oracle.SEED_RANDOM, 2, 1)
    prev = None
    for _ in range(30):
        before = {s: g.particles(s) for s in (0, 1)}
        assert g.step(1) == oracle.OK
        after = {s: g.particles(s) for s in (0, 1)}
        # energy before emission of each pushed lepton = gamma(p_old + q E0 dt)
        e_pushed = 0.0
        for s, q in ((0, -1.0), (1, 1.0)):
            pn = before[s]["p"] + q * e0 * dt
            e_pushed += np.sum(np.sqrt(1 + pn * pn))
        e_after = sum(np.sum(np.sqrt(1 + after[s]["p"] ** 2)) for s in (0, 1))
        tot = e_after
        assert abs(tot - e_pushed) <= 1e-9 * e_pushed
        prev = tot
    assert prev is not None and g.count(0) > 2


def test_invalid_parameters_rejected():
    base = dict(n_cells=16, dx=1.0, dt=0.45, boundary=0, e0=1.0, gamma_thr=100.0, f=0.5,
                l_gamma=0.0, weight=1.0, seed=1)
    assert oracle.validate(**base) == oracle.OK
    for k, v in [("dt", 1.0), ("dt", 1.5), ("f", 0.01), ("f", 1.0), ("gamma_thr", 1.0),
                 ("n_cells", 1), ("boundary", 7), ("l_gamma", -1.0), ("weight", -1.0),
                 ("e0", float("nan")), ("n_cells", 2**22 + 1), ("l_gamma", 1e6),
                 ("l_gamma", 1e30)]:
        assert oracle.validate(**{**base, k: v}) == oracle.ERR_ARG, k
    # positions on the 2^-24 grid of the mixed path leave room for longer paths
    assert oracle.validate(**{**base, "l_gamma": 1e6, "precision": oracle.MIXED}) == oracle.OK


# -------------------------------------------------------- analytic physics
@pytest.mark.parametrize("f,steps", [(0.1, 560), (0.01, 2300)])
def test_frozen_field_growth_rate_matches_population_model(f, steps):
    """Section 3: in a uniform field the cascade grows as exp(Gamma t) with
    Gamma the root of Eqs. 1-2 (Gamma t_a -> W(2/f) for small f)."""
    gthr, e0 = 500.0, 1.0
    ta = gthr / e0
    dt = 0.1 * f * ta          # t_p / dt = 10
    g = oracle.OracleGap(n_cells=4, dx=2 * dt, dt=dt, boundary=oracle.PERIODIC, e0=e0,
                         gamma_thr=gthr, f=f, l_gamma=0.0, weight=0.0, seed=1)
    g.seed(oracle.SEED_RANDOM, 1, 1)
    assert g.step(steps) == oracle.OK
    h = g.history()
    n = h["n_minus"].astype(float)
    t = (h["step"] + 1) * dt
    sel = t > 1.5 * ta
    G = np.polyfit(t[sel], np.log(n[sel]), 1)[0]
    exact = A.growth_rate_exact(f, ta)
    assert abs(G / exact - 1.0) < 0.10, (G, exact)
    # the Lambert form of Eq. 3 is the small-f limit of the same root
    assert abs(A.growth_rate_lambert(f, ta) / exact - 1.0) < 0.05


@pytest.fixture(scope="module")
def screening_run():
    """Self-consistent, resolved screening run: periodic, in-place pairs,
    f = 0.1, t_p/dt = 10, ~300 macros per cell per species at n_s."""
    f, e0, gthr, dt, dx, nc = 0.1, 100.0, 100.0, 0.01, 0.1, 40
    ns = A.screening_density(e0, gthr, f)
    w = ns * dx / 300.0
    g = oracle.OracleGap(n_cells=nc, dx=dx, dt=dt, boundary=oracle.PERIODIC, e0=e0,
                         gamma_thr=gthr, f=f, l_gamma=0.0, weight=w, seed=7)
    g.seed(oracle.SEED_RANDOM, nc, 1)
    snaps = []
    for _ in range(240):
        assert g.step(5) == oracle.OK
        P = np.concatenate([g.particles(0)["p"], g.particles(1)["p"]])
        gam = np.sqrt(1 + P * P)
        snaps.append((g.steps_done - 1, gam.mean(), np.mean(gam ** -3.0)))
    return dict(g=g, h=g.history(), snaps=np.array(snaps), f=f, e0=e0, gthr=gthr, dt=dt,
                dx=dx, nc=nc, w=w, ns=ns)


def test_screening_density_eq5(screening_run):
    """Eq. 5 overestimates the density at screening by a factor 1.5-2."""
    r = screening_run
    h = r["h"]
    i_s = int(np.argmax(h["e_mean"] < 0))
    assert i_s > 0
    n_at_s = h["n_minus"][i_s] * r["w"] / (r["nc"] * r["dx"])
    ratio = n_at_s / r["ns"]
    assert 0.35 <= ratio <= 1.0, ratio


def test_energy_balance_and_mean_gamma(screening_run):
    """Section 4: at screening the field energy E0^2/8pi has gone to the
    leptons, n_s <gamma> m c^2 = E0^2/8pi, with <gamma> ~ gamma_thr/ln(2/f)."""
    r = screening_run
    h = r["h"]
    i_s = int(np.argmax(h["e_mean"] < 0))
    field0 = r["e0"] ** 2 / 2 * r["nc"] * r["dx"]
    assert abs(h["kinetic"][i_s] / field0 - 1.0) < 0.25
    snaps = r["snaps"]
    j = int(np.argmin(np.abs(snaps[:, 0] - i_s)))
    assert abs(snaps[j, 1] / A.mean_gamma(r["gthr"], r["f"]) - 1.0) < 0.25


def test_oscillation_frequency_relativistic(screening_run):
    """Section 5: after screening <E> oscillates at omega_0 = sqrt(2 n <1/gamma^3>)
    (normalised), with n and <1/gamma^3> measured from the particles."""
    r = screening_run
    h = r["h"]
    Em = h["e_mean"]
    zc = np.where(np.diff(np.sign(Em)) != 0)[0]
    assert len(zc) >= 5
    # two full periods after the first reversal
    a, b = zc[0], zc[4]
    omega_meas = 2 * 2 * math.pi / ((b - a) * r["dt"])
    snaps = r["snaps"]
    sel = (snaps[:, 0] >= a) & (snaps[:, 0] < b)
    inv_g3 = snaps[sel, 2].mean()
    n = h["n_minus"][a:b].mean() * r["w"] / (r["nc"] * r["dx"])
    omega_th = A.relativistic_plasma_frequency(n, inv_g3)
    assert abs(omega_meas / omega_th - 1.0) < 0.15, (omega_meas, omega_th)


def test_energy_conserved_in_resolved_run(screening_run):
    """Total energy (leptons, field, photons, losses) drifts by well under 1%
    in the resolved run (leapfrog error only)."""
    h = screening_run["h"]
    tot = h["kinetic"] + h["field"] + h["photon_energy"] + h["lost_energy"]
    assert np.max(np.abs(tot / tot[0] - 1.0)) < 1e-2


# ---------------------------------------------------------- co-rotating frame
def _corot(n_cells, precision, boundary, dt=1e-2, ppc=8):
    import workloads
    from tests import pic_cases as pc
    cfg = workloads.corotating_gap(n_cells=n_cells, dx=0.1, dt=dt, ppc_plus=ppc, gamma_thr=1e30,
                                   f=0.5, precision=precision, capacity=0)
    cfg["boundary"] = boundary
    return cfg, pc.make_oracle(cfg)


def test_imposed_current_closed_form():
    """Section 7: with no plasma, Ampere's law dE/dt = -(J - j_m) gives
    E(t) = E0 + j_m t in every cell (each step adds j_m dt once)."""
    g = oracle.OracleGap(n_cells=16, dx=0.1, dt=1e-3, boundary=oracle.ABSORBING, e0=0.25,
                         gamma_thr=1e30, f=0.5, l_gamma=0.0, weight=1.0, seed=3, j_m=1.5)
    n = 1000
    assert g.step(n) == 0
    E = g.fields()["E"]
    exact = 0.25 + n * (1.5 * 1e-3)
    assert np.all(np.abs(E - exact) <= n * np.spacing(exact))
    assert np.all(E == E[0])


@pytest.mark.parametrize("precision,K,eps", [(oracle.FP64, 40, 2.0**-52), (oracle.MIXED, 24, 2.0**-23)])
def test_corotating_loading_is_an_equilibrium(precision, K, eps):
    """Section 7: electrons at -2 rho_GJ and positrons at rho_GJ satisfy Gauss's
    law dE/dx = rho - rho_GJ with E = 0, and cold streams with J = j_m satisfy
    Ampere's law, so in a periodic domain E stays zero up to the rounding of
    the displacement (2^-K cell per step, against |v| dt/dx = 0.05 cell) and of
    v = p / gamma; Gauss's law with the background holds exactly."""
    n = 500
    cfg, g = _corot(400, precision, oracle.PERIODIC)
    assert g.step(n) == 0
    F = g.fields()
    E, rho = F["E"], F["rho"]
    jmdt = 1.5 * cfg["dt"]
    rel = 2.0**-K / (0.5 * cfg["dt"] / cfg["dx"]) + 8 * eps
    assert np.max(np.abs(E)) <= n * jmdt * rel, (np.max(np.abs(E)), n * jmdt * rel)
    resid = (E - np.roll(E, 1)) - (rho[:-1] - cfg["rho_gj"] * cfg["dx"])
    assert np.max(np.abs(resid)) <= 16 * 2.0**-52 * max(np.max(np.abs(E)), 1.0)


def test_corotating_gap_opens_at_the_walls():
    """Section 7: with open walls the field stays zero everywhere except near
    the walls, where streams leave the domain uncompensated and gaps open; the
    interior keeps rho = rho_GJ and J = j_m."""
    cfg, g = _corot(1000, oracle.FP64, oracle.ABSORBING)
    assert g.step(300) == 0
    F = g.fields()
    E, rho = F["E"], F["rho"]
    assert abs(E[0]) > 0.5 and abs(E[-1]) > 0.5
    assert np.max(np.abs(E[300:700])) < 1e-9
    resid = (E[1:] - E[:-1]) - (rho[1:-1] - cfg["rho_gj"] * cfg["dx"])
    assert np.max(np.abs(resid)) <= 64 * 2.0**-52 * max(np.max(np.abs(E)), 1.0)


# ------------------------------------------------------------ pair-event map
def test_event_map_single_emitter_closed_form():
    """One positron with p = 1000 in zero field (w = 0, pairs in place): at step
    0 it moves v dt / dx cells and, at or above gamma_thr = 100 with
    gamma_pair = 50, makes k = floor((gamma - gamma_thr) / gamma_pair) + 1
    pairs in the cell it reached; its children (gamma' = 25) and itself (now
    below threshold) make none afterwards."""
    g = oracle.OracleGap(n_cells=64, dx=1.0, dt=0.45, boundary=oracle.PERIODIC, e0=0.0,
                         gamma_thr=100.0, f=0.5, l_gamma=0.0, weight=0.0, seed=11)
    g.seed_explicit(1, [40], [0.75], [1000.0], [7])
    g.event_map(16, 1, 10)
    assert g.step(10) == 0
    m = g.read_event_map()
    gamma = math.sqrt(1.0 + 1000.0**2)
    k = int((gamma - 100.0) // 50.0) + 1
    x1 = 40 + 0.75 + 1000.0 / gamma * 0.45  # position after the move, cells
    assert m.sum() == k
    assert m[0, int(x1) * 16 // 64] == k
    assert m[1:].sum() == 0


def test_event_map_rows_match_history():
    """Summed over cells, each row of the event map is the number of pairs the
    history records for the steps of that row."""
    g = oracle.OracleGap(n_cells=512, dx=1.0, dt=0.45, boundary=oracle.ABSORBING, e0=50.0,
                         gamma_thr=100.0, f=0.5, l_gamma=20.0, weight=1.0, seed=2012055871)
    g.seed(oracle.SEED_RANDOM, 256, 1)
    g.event_map(32, 25, 20)
    assert g.step(500) == 0
    m = g.read_event_map()
    h = g.history()
    made = np.diff(np.concatenate([[0], h["pairs_created"]]))
    assert made.sum() > 1000
    assert np.array_equal(m.sum(axis=1), made.reshape(20, 25).sum(axis=1))


# ------------------------------------------------- non-uniform field and seed
LAM, E_SURF = 64.0, 2.0  # E(x) = E_SURF exp(-x / LAM) at the cell centres


def _exp_field_gap(r, gamma_thr=1e300, precision=oracle.FP64, weight=0.0, n_cells=256,
                   shape=oracle.SHAPE_LINEAR):
    """Gap of n_cells/dx = 256 length units, dx = 1/r, dt = 0.4/r, with the
    decaying field sampled at the cell centres (x = (c + 1/2) dx); absorbing
    walls, or periodic for the quadratic shape (the lepton stays far from
    the ends either way)."""
    dx, dt = 1.0 / r, 0.4 / r
    nc = n_cells * r
    bc = oracle.ABSORBING if shape == oracle.SHAPE_LINEAR else oracle.PERIODIC
    g = oracle.OracleGap(n_cells=nc, dx=dx, dt=dt, boundary=bc, e0=0.0,
                         gamma_thr=gamma_thr, f=0.5, l_gamma=0.0, weight=weight, seed=1,
                         precision=precision, shape=shape)
    g.set_fields(E_SURF * np.exp(-(np.arange(nc) + 0.5) * dx / LAM))
    return g, dx, dt


def _put(g, species, x0, dx, pid):
    c = int(x0 / dx)
    g.seed_explicit(species, [c], [x0 / dx - c], [0.0], [pid])


def _energy_error(r, precision=oracle.FP64, T=100.0, x0=20.0, shape=oracle.SHAPE_LINEAR):
    """Positron from rest at x0: in a static field gamma(x) = 1 + q (phi(x0) -
    phi(x)) = 1 + E_SURF LAM (exp(-x0/LAM) - exp(-x/LAM)).  p^{n+1/2} is
    compared at the midpoint of x^n and x^{n+1}."""
    g, dx, dt = _exp_field_gap(r, precision=precision, shape=shape)
    _put(g, 1, x0, dx, 3)
    n = int(round(T / dt))
    assert g.step(n - 1) == oracle.OK
    P = g.particles(1)
    xa = (P["cell"][0] + P["off"][0]) * dx
    assert g.step(1) == oracle.OK
    P = g.particles(1)
    xm = 0.5 * (xa + (P["cell"][0] + P["off"][0]) * dx)
    exact = 1.0 + E_SURF * LAM * (math.exp(-x0 / LAM) - math.exp(-xm / LAM))
    return math.sqrt(1.0 + P["p"][0] ** 2) - exact


@pytest.mark.parametrize("shape", [oracle.SHAPE_LINEAR, oracle.SHAPE_QUADRATIC])
def test_nonuniform_field_energy_gain_second_order(shape):
    """Energy gained in the decaying field against the potential drop: the
    node-averaged gather (linear or spline) and the leapfrog are second
    order, so the error falls by 4 per halving of dx and dt (a gather
    displaced by a fraction of a cell would make it first order)."""
    errs = [_energy_error(r, shape=shape) for r in (1, 2, 4, 8)]
    assert abs(errs[0]) < 0.05
    for a, b in zip(errs[:-1], errs[1:]):
        assert 3.8 < a / b < 4.2, errs
    # binary32 particles: same error until its round-off (p ~ 100, 2^-24)
    for r in (1, 2):
        assert abs(_energy_error(r, oracle.MIXED, shape=shape) - errs[r // 2]) < 2e-3


@pytest.mark.parametrize("species,x0", [(1, 10.0), (1, 60.0), (0, 60.0), (1, 100.0)])
def test_nonuniform_field_first_emission_matches_ode(species, x0):
    """First emission of a lepton released at rest in the decaying field
    against the equations of motion dp/dt = q E(x), dx/dt = p / gamma solved
    by scipy (rtol 1e-11): emission at the first step whose p^{n+1/2} has
    gamma >= gamma_thr.  A positron at x0 = 100 sees a potential drop of only
    E_SURF LAM exp(-100/LAM) = 27 < gamma_thr - 1 ahead of it and never emits."""
    from scipy.integrate import solve_ivp
    gthr, r = 40.0, 4
    g, dx, dt = _exp_field_gap(r, gamma_thr=gthr)
    _put(g, species, x0, dx, 5)
    steps = 3000
    assert g.step(steps) == oracle.OK
    h = g.history()
    fired = np.nonzero(h["photons_emitted"] > 0)[0]
    q = 1.0 if species == 1 else -1.0
    L = 256.0

    def rhs(t, y):
        x = min(max(y[0], 0.0), L)
        return [y[1] / math.sqrt(1.0 + y[1] ** 2), q * E_SURF * math.exp(-x / LAM)]

    def reach(t, y):
        return math.sqrt(1.0 + y[1] ** 2) - gthr
    reach.terminal = True

    def wall(t, y):
        return y[0] * (L - y[0])
    wall.terminal = True
    sol = solve_ivp(rhs, (0.0, steps * dt), [x0, 0.0], events=(reach, wall), rtol=1e-11,
                    atol=1e-12)
    if len(sol.t_events[0]) == 0:
        assert fired.size == 0, fired[:3]
        return
    # p^{n+1/2} is the momentum at (n + 1) dt after release at rest
    t_star = sol.t_events[0][0]
    assert fired.size > 0
    assert abs(fired[0] - (t_star / dt - 1.0)) <= 1.5, (fired[0], t_star / dt - 1.0)


@pytest.mark.parametrize("precision", [oracle.FP64, oracle.MIXED])
def test_gauss_residual_with_nonuniform_start(precision):
    """A decaying initial field implies a fixed background charge dE/dx; the
    deposit keeps E_c - E_{c-1} - (E0_c - E0_{c-1}) = rho_c - rho0_c on the
    interior nodes at round-off, with a non-uniform seed and a cascade."""
    import workloads
    cfg = workloads.nonuniform_gap(n_cells=512, length=512.0, dt=0.45, seed_pairs=256,
                                   seed_scale=0.1, e0=50.0, gamma_thr=100.0, f=0.5,
                                   l_gamma=20.0, weight=1.0, precision=precision,
                                   capacity=100_000, photon_capacity=100_000)
    from tests.pic_cases import make_oracle
    g = make_oracle(cfg)
    F0 = g.fields()
    assert g.step(400) == oracle.OK
    assert g.history()["pairs_created"][-1] > 1000
    F = g.fields()
    E, rho = F["E"], F["rho"]
    dE = (E[1:] - E[:-1]) - (F0["E"][1:] - F0["E"][:-1])
    r = dE - (rho[1:-1] - F0["rho"][1:-1])
    # 400 binary64 field updates of values below 50
    assert np.max(np.abs(r)) < 400 * 50.0 * 2.0**-52


# ------------------------------------------------------- spread of gamma_thr
def test_threshold_spread_first_emissions_are_uniform():
    """Leptons released at rest in a frozen uniform field reach gamma ~
    E0 dt (n + 1) at step n, so each one's first emission marks its own
    threshold.  With a spread sigma the thresholds are uniform in
    gamma_thr (1 - sigma, 1 + sigma): no emission before gamma_thr (1 - sigma),
    and first emissions spread evenly over the steps (chi-square over 18 bins,
    within the window before any lepton emits a second time and before any
    child reaches threshold)."""
    e0, dt, gthr, f, sigma = 1.0, 0.5, 1000.0, 0.5, 0.3
    g = oracle.OracleGap(n_cells=64, dx=1.0, dt=dt, boundary=oracle.PERIODIC, e0=e0,
                         gamma_thr=gthr, f=f, l_gamma=0.0, weight=0.0, seed=2012055871,
                         gamma_thr_spread=sigma)
    n_pairs = 10000
    g.seed(oracle.SEED_RANDOM, n_pairs, 1)
    # p^{n+1/2} = (n + 1) E0 dt: step n passes the thresholds in (gamma_{n-1}, gamma_n]
    # with gamma_n = sqrt(1 + ((n + 1) E0 dt)^2); the first step whose gamma
    # reaches the lowest threshold gamma_thr (1 - sigma)
    lo = next(n for n in range(10**6)
              if math.sqrt(1.0 + ((n + 1) * e0 * dt) ** 2) >= gthr * (1 - sigma))
    hi = lo + 900                              # a child needs 900 steps to reach it
    assert g.step(hi) == oracle.OK
    em = np.diff(g.history()["photons_emitted"], prepend=0)
    assert em[:lo].sum() == 0 and em[lo] > 0
    n = np.arange(lo, hi)
    gam = np.sqrt(1.0 + ((n + 1) * e0 * dt) ** 2) - np.sqrt(1.0 + (n * e0 * dt) ** 2)
    expect = (2 * n_pairs * gam / (2 * sigma * gthr)).reshape(18, 50).sum(axis=1)
    counts = em[lo:hi].reshape(18, 50).sum(axis=1)
    chi2 = float(((counts - expect) ** 2 / expect).sum())
    assert chi2 < 42.3, (chi2, counts, expect)  # 99.9% point of chi2 with 18 dof


def test_threshold_spread_validation():
    """sigma in [0, 1), and the lowest threshold minus gamma_pair keeps gamma >= 1."""
    base = dict(n_cells=8, dx=1.0, dt=0.5, boundary=oracle.PERIODIC, e0=1.0, gamma_thr=100.0,
                f=0.5, l_gamma=0.0, weight=1.0, seed=1)
    assert oracle.validate(**base, gamma_thr_spread=0.0) == oracle.OK
    assert oracle.validate(**base, gamma_thr_spread=0.49) == oracle.OK
    for bad in (-0.1, 0.5, 1.0, float("nan")):
        assert oracle.validate(**base, gamma_thr_spread=bad) == oracle.ERR_ARG, bad


# ------------------------------------------------------ quadratic particle shape
@pytest.mark.parametrize("precision", [oracle.FP64, oracle.MIXED])
@pytest.mark.parametrize("cell,off", [(5, 0.0), (5, 0.25), (5, 0.5), (5, 0.75), (5, 0.999),
                                      (0, 0.1), (15, 0.9)])
def test_quadratic_shape_charge_of_one_lepton(precision, cell, off):
    """One positron at x = cell + off (weight dx): nodes j-1, j, j+1 around the
    nearest node j = floor(x + 1/2) hold (1/2 - d)^2/2, 3/4 - d^2,
    (1/2 + d)^2/2 with d = x - j, to 3 units of 2^-K (the outer two rounded
    down, the offset on its grid), the others nothing; periodic folding at
    both ends; the total is exactly one charge."""
    N = 16
    g = oracle.OracleGap(n_cells=N, dx=1.0, dt=0.5, boundary=oracle.PERIODIC, e0=0.0,
                         gamma_thr=1e300, f=0.5, l_gamma=0.0, weight=1.0, seed=1,
                         precision=precision, shape=oracle.SHAPE_QUADRATIC)
    g.seed_explicit(1, [cell], [off], [0.0], [3])
    rho = g.fields()["rho"]
    x = cell + off
    j = math.floor(x + 0.5)
    d = x - j
    expect = np.zeros(N)
    for k, v in ((j - 1, 0.5 * (0.5 - d) ** 2), (j, 0.75 - d * d), (j + 1, 0.5 * (0.5 + d) ** 2)):
        expect[k % N] += v
    assert np.max(np.abs(rho[:N] - expect)) <= 3 * 2.0 ** -g.offset_bits
    assert rho[N] == rho[0] and rho[:N].sum() == 1.0


@pytest.mark.parametrize("boundary", [oracle.PERIODIC, oracle.ABSORBING])
@pytest.mark.parametrize("precision", [oracle.FP64, oracle.MIXED])
def test_gauss_residual_quadratic_shape(precision, boundary):
    """The spline deposit conserves charge exactly: E_c - E_{c-1} = rho_c at
    every node (every interior node with absorbing walls) at round-off,
    through a cascade with photons, and with absorbing walls through the
    removal of the leptons that leave (carried 3/2 cells past the wall)."""
    g = oracle.OracleGap(n_cells=128, dx=1.0, dt=0.45, boundary=boundary, e0=20.0,
                         gamma_thr=60.0, f=0.5, l_gamma=8.0, weight=0.5, seed=11,
                         precision=precision, shape=oracle.SHAPE_QUADRATIC)
    g.seed(oracle.SEED_RANDOM, 256, 1)
    steps = 300
    assert g.step(steps) == oracle.OK
    F = g.fields()
    E, rho = F["E"], F["rho"]
    if boundary == oracle.PERIODIC:
        r = (E - np.roll(E, 1)) - rho[:-1]
    else:
        r = (E[1:] - E[:-1]) - rho[1:-1]
        h = g.history()
        assert h["absorbed_minus"][-1] > 100 and h["absorbed_plus"][-1] > 100
    assert np.abs(r).max() <= 10 * np.finfo(float).eps * steps * np.abs(E).max()
    assert g.history()["pairs_created"][-1] > 256


def test_quadratic_shape_heats_an_unresolved_plasma_less():
    """A cold pair plasma whose Debye length is far below the cell (v_th =
    0.05 c, n = 1 per species, dx = 1, dt = 0.45) heats numerically; the
    spline's smoother deposit and gather cut the heating over 2000 steps by
    more than five times against the linear shape."""
    def drift(shape):
        N = 256
        g = oracle.OracleGap(n_cells=N, dx=1.0, dt=0.45, boundary=oracle.PERIODIC, e0=0.0,
                             gamma_thr=1e300, f=0.5, l_gamma=0.0, weight=0.05, seed=9,
                             shape=shape)
        rng = np.random.default_rng(3)
        n = N * 20
        X = rng.random(n) * N
        cell = np.floor(X).astype(np.int32)
        for sp in (0, 1):
            g.seed_explicit(sp, cell, X - cell, rng.normal(0.0, 0.05, n),
                            np.arange(n, dtype=np.uint64) * 2 + sp)
        assert g.step(2000) == oracle.OK
        h = g.history()
        W = h["kinetic"] + h["field"]
        return W[-1] / W[0] - 1.0
    lin, quad = drift(oracle.SHAPE_LINEAR), drift(oracle.SHAPE_QUADRATIC)
    assert lin > 0.05 and 0.0 < quad < lin / 5.0, (lin, quad)


def test_quadratic_shape_validation():
    """The spline needs at least four cells."""
    base = dict(dx=1.0, dt=0.5, e0=1.0, gamma_thr=100.0, f=0.5, l_gamma=0.0, weight=1.0, seed=1)
    assert oracle.validate(n_cells=8, boundary=oracle.PERIODIC, shape=1, **base) == oracle.OK
    assert oracle.validate(n_cells=8, boundary=oracle.ABSORBING, shape=1, **base) == oracle.OK
    assert oracle.validate(n_cells=3, boundary=oracle.PERIODIC, shape=1, **base) == oracle.ERR_ARG
    assert oracle.validate(n_cells=8, boundary=oracle.PERIODIC, shape=2, **base) == oracle.ERR_ARG


def test_quadratic_shape_lepton_leaving_through_a_wall():
    """A positron driven out through the right wall: Gauss's law, counted
    from the initial field and charge, holds on every interior node at every
    step; once the positron has left, no interior node holds any charge (its
    charge went out through the last cells as current)."""
    N = 16
    g = oracle.OracleGap(n_cells=N, dx=1.0, dt=0.45, boundary=oracle.ABSORBING, e0=5.0,
                         gamma_thr=1e300, f=0.5, l_gamma=0.0, weight=1.0, seed=1,
                         shape=oracle.SHAPE_QUADRATIC)
    g.seed_explicit(1, [N - 3], [0.5], [0.0], [3])
    F0 = g.fields()
    E0, rho0 = F0["E"].copy(), F0["rho"].copy()
    assert rho0[1:-1].sum() == 1.0
    left_at = None
    for n in range(40):
        assert g.step(1) == oracle.OK
        F = g.fields()
        r = (F["E"][1:] - F["E"][:-1]) - (E0[1:] - E0[:-1]) - (F["rho"][1:-1] - rho0[1:-1])
        assert np.abs(r).max() < 1e-12, (n, r)
        if g.count(1) == 0 and left_at is None:
            left_at = n
            assert np.all(F["rho"][1:-1] == 0.0)
    assert left_at is not None and g.history()["absorbed_plus"][-1] == 1
