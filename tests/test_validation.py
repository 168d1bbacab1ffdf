"""The HIP path at the paper's scale against the analytic results of
sections 3-6 (arXiv:2012.05587).

Setup of section 3: a seed pair plasma at rest in a uniform field E0,
periodic, pairs made in place.  2000 cells over L = 10^1.5 c/omega_p0,
dt = 10^-3.5, E0 = 10^3.5, gamma_thr = 500, 2000 seed pairs of weight dx
(seed density 1 per species).  The cascade grows to 1e7-1e8 leptons per
species, so only the GPU runs it; the oracle's pins cover the same
relations at small scale.

Measured against:
- energy: field + kinetic stays constant (pairs made in place lose nothing);
- section 3: growth rate (exact root of Eqs. 1-2), screening time t_s, the
  screening density of Eq. 5, which the paper finds to overestimate the
  density at the end of the cascade;
- section 4: the exponential spectrum of Eq. 8 and its mean, Eq. 10, at
  screening;
- section 5: each half period of the large-amplitude oscillation of <E>
  against omega_0^2 = 2 n <1/gamma^3> (normalised), with n and
  <1/gamma^3> measured on the device over that half period;
- section 6 (f = 0.1): secondary bursts once per cycle near <E> = 0, and
  the damping of the oscillation amplitude fitted by Eq. 24;
- the non-uniform start of the conclusion (field and seed decaying with
  altitude): screening at each altitude on the local clock of section 3;
- a spread of the threshold (also named in the conclusion): growth, omega_0,
  and the smoothing it brings to the generations and the bursts;
- the co-rotating gap of section 7 at the paper's scale: equilibrium bulk,
  the gap at one wall, the first pairs once its potential drop exceeds
  gamma_thr, and the screening by the bursts.

f = 10^-3 (the smallest f the paper reports checking) needs f gamma_thr >= 2
for a pair to hold two rest masses, so it runs with gamma_thr = 5000.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import analytic as A

pytestmark = pytest.mark.gpu

SAMPLE = 50      # steps between <1/gamma^3> samples
P_RANGE = 64.0   # momentum range of the <1/gamma^3> histogram
P_BINS = 8192
# (f, precision, gamma_thr, steps, shape): the steps cover screening and at
# least four half periods of the oscillation (ten for f = 0.1 in mixed
# precision); shape 1 is the quadratic spline, which at this resolution must
# give the same physics as the linear shape
CASES = [(0.1, workloads.MIXED, 500.0, 12000, 0), (0.03, workloads.MIXED, 500.0, 4800, 0),
         (0.01, workloads.MIXED, 500.0, 4800, 0), (0.1, workloads.FP64, 500.0, 7600, 0),
         (0.001, workloads.MIXED, 5000.0, 44000, 0), (0.1, workloads.MIXED, 500.0, 12000, 1)]


def _spectrum(g):
    """Counts of both species in 1000 momentum bins over [-1000, 1000]."""
    return sum(g.phase_space(sp, 1, 1000, -1000.0, 1000.0)[0] for sp in (0, 1))


def _inv_gamma3(g):
    """<1/gamma^3> over both species from device histograms of p in
    [-P_RANGE, P_RANGE].  The two edge bins also hold the leptons outside the
    range, whose 1/gamma^3 < 4e-6, and are counted with weight 0."""
    dp = 2.0 * P_RANGE / P_BINS
    pc = -P_RANGE + (np.arange(P_BINS) + 0.5) * dp
    w = (1.0 + pc * pc) ** -1.5
    w[0] = w[-1] = 0.0
    num = den = 0.0
    for sp in (0, 1):
        h = g.phase_space(sp, 1, P_BINS, -P_RANGE, P_RANGE)[0].astype(np.float64)
        num += float(h @ w)
        den += float(h.sum())
    return num / den if den else float("nan")


def run_uniform_cascade(f, precision, gamma_thr, steps, spread=0.0, shape=0):
    """Runs the section 3 setup on the GPU; returns the configuration, the
    history and the sampled <1/gamma^3>."""
    import torch

    import paper_2012_05587_amd as P
    from tests.pic_cases import gpu_params
    cfg = workloads.uniform_cascade(f, gamma_thr=gamma_thr, precision=precision,
                                    gamma_thr_spread=spread, shape=shape)
    g = P.Gap(gpu_params(cfg, history_rows=steps + 8, diag_every=1),
              stream=torch.cuda.Stream())
    try:
        g.seed_particles(cfg["seed_mode"], cfg["n_pairs"], cfg["macro_per_pair"])
        samples, spectra = [], []
        done = 0
        while done < steps:
            k = min(SAMPLE, steps - done)
            g.step_n(k)
            done += k
            samples.append((done - 1, _inv_gamma3(g)))
            spectra.append(_spectrum(g))
        h = g.read_history()
    finally:
        g.close()
        del g
        torch.cuda.empty_cache()
    return cfg, h, np.array(samples), np.array(spectra)


def spectrum_fit(cfg, samples, spectra, step):
    """Eq. 8 at the sample nearest `step`: a line through ln(counts) against
    gamma over [0.15, 0.85] gamma_thr (|p| bins, both signs and species), its
    slope times gamma_thr, R^2, and the mean gamma of the binned leptons."""
    j = int(np.argmin(np.abs(samples[:, 0] - step)))
    h = spectra[j].astype(np.float64)
    edges = np.linspace(-1000.0, 1000.0, 1001)
    gam = np.sqrt(1.0 + (0.5 * (edges[1:] + edges[:-1])) ** 2)
    hp, g = h[500:] + h[:500][::-1], gam[500:]
    gthr = cfg["gamma_thr"]
    sel = (g > 0.15 * gthr) & (g < 0.85 * gthr) & (hp > 0)
    y = np.log(hp[sel])
    a = np.polyfit(g[sel], y, 1)
    r = y - np.polyval(a, g[sel])
    return dict(slope=float(a[0] * gthr), r2=float(1.0 - (r @ r) / ((y - y.mean()) @ (y - y.mean()))),
                mean_gamma=float((hp * g).sum() / hp.sum()), step=int(samples[j, 0]))


def measure(cfg, h, samples):
    f, dt, e0, gthr = cfg["f"], cfg["dt"], cfg["e0"], cfg["gamma_thr"]
    L = cfg["n_cells"] * cfg["dx"]
    w = cfg["weight"]
    t = (h["step"] + 1) * dt
    n = h["n_minus"].astype(np.float64) * w / L            # density per species
    W = h["kinetic"] + h["field"] + h["photon_energy"] + h["lost_energy"]
    W0 = e0 * e0 / 2.0 * L + 2.0 * cfg["n_pairs"] * w      # field plus rest mass of the seed
    ta = A.t_accel(e0, gthr)
    G_exact = A.growth_rate_exact(f, ta)
    sel = (t > ta) & (t < 3.0 * ta)
    G = float(np.polyfit(t[sel], np.log(h["n_minus"][sel].astype(np.float64)), 1)[0])
    i_s = int(np.argmax(h["e_mean"] < 0.0))
    n0 = cfg["n_pairs"] * w / L
    ts_formula = A.screening_time(e0, n0, G_exact)
    ns = A.screening_density(e0, gthr, f)
    gmean = h["kinetic"] / (w * (h["n_minus"] + h["n_plus"]).astype(np.float64))
    # half periods of <E> after screening
    em = h["e_mean"]
    pc = h["pairs_created"].astype(np.float64)
    rate = np.convolve(np.diff(pc, prepend=pc[0]), np.ones(51) / 51.0, mode="same")
    zc = np.nonzero(np.sign(em[i_s:-1]) != np.sign(em[i_s + 1:]))[0] + i_s
    zc = np.concatenate([[i_s - 1], zc])  # i_s is the first step with <E> < 0
    half = []
    for a, b in zip(zc[:-1], zc[1:]):
        m = (samples[:, 0] > a) & (samples[:, 0] <= b)
        if m.sum() < 3:
            continue
        ig3 = float(np.mean(samples[m, 1]))
        nm = float(np.mean(n[a:b + 1]))
        half.append(dict(a=int(a), b=int(b), omega=math.pi / ((b - a) * dt),
                         omega_th=A.relativistic_plasma_frequency(nm, ig3), inv_g3=ig3,
                         amp=float(np.max(np.abs(em[a:b + 1]))), pairs=float(pc[b] - pc[a]),
                         burst_at=float((np.argmax(rate[a:b]) + 0.5) / (b - a))))
    return dict(
        f=f, energy_drift=float(np.max(np.abs(W / W0 - 1.0))),
        G=G, G_exact=G_exact, i_s=i_s, t_s=float(t[i_s]), t_s_formula=ts_formula, t_a=ta,
        growth_s=float(h["n_minus"][i_s] / cfg["n_pairs"]),
        kinetic_over_W0=float(h["kinetic"][i_s] / W0), n_s=float(n[i_s]), n_s_eq5=ns,
        gmean_s=float(gmean[i_s]), gmean_eq10=A.mean_gamma(gthr, f),
        inv_g3_exp=math.log(2.0 / f) / (2.0 * gthr), half_periods=half)


def damping_fit(half, cycles):
    """Eq. 24 with the residual term dropped: the amplitude of <E> decays as
    exp(-eps0 omega0 t / (4 pi)), i.e. by a factor 1 - eps0/2 per cycle.
    Fits eps0 to the amplitudes of the first 2 * cycles half periods, and
    measures eps, the jump of omega^2 per cycle that the jump conditions of
    section 6 call eps_n, from the half-period frequencies."""
    hp = half[:2 * cycles]
    tc = np.array([(x["a"] + x["b"]) / 2.0 for x in hp])
    amp = np.array([x["amp"] for x in hp])
    om = np.array([x["omega"] for x in hp])
    slope = np.polyfit(tc, np.log(amp), 1)[0]        # per step
    om2 = np.polyfit(tc, np.log(om * om), 1)[0]      # per step
    steps_per_cycle = 2.0 * (hp[-1]["b"] - hp[0]["a"]) / len(hp)
    return dict(eps0_fit=float(-2.0 * slope * steps_per_cycle),
                eps_omega=float(om2 * steps_per_cycle), omega0=float(np.mean(om)),
                amp_loss_per_cycle=float(1.0 - math.exp(slope * steps_per_cycle)))


def _id(case):
    f, p, gthr, _, shape = case
    return (f"f{f}-{'fp64' if p == workloads.FP64 else 'mixed'}-g{int(gthr)}"
            + ("-spline" if shape else ""))


@pytest.mark.parametrize("case", CASES, ids=[_id(c) for c in CASES])
def test_uniform_cascade_at_paper_scale(case):
    f, precision, gthr, steps, shape = case
    cfg, h, samples, spectra = run_uniform_cascade(f, precision, gthr, steps, shape=shape)
    r = measure(cfg, h, samples)
    print({k: v for k, v in r.items() if k != "half_periods"})
    for x in r["half_periods"]:
        print(x)
    assert len(h) == steps and h["step"][-1] == steps - 1
    # pairs made in place conserve field plus kinetic energy up to the scheme's error
    assert r["energy_drift"] < 2e-3, r["energy_drift"]
    # at screening nearly all the field energy sits in the leptons
    assert r["kinetic_over_W0"] > 0.98, r["kinetic_over_W0"]
    if f >= 0.01:
        # section 3: growth over [t_a, 3 t_a] (two generations) against Eqs. 1-2
        assert abs(r["G"] / r["G_exact"] - 1.0) < 0.08, (r["G"], r["G_exact"])
        # screening: the first sign change of <E>, against t_s of section 3
        # (exponential growth from t = 0, so the first generation's delay of
        # about t_a makes the measured time longer)
        assert 1.0 < r["t_s"] / r["t_s_formula"] < 1.3, (r["t_s"], r["t_s_formula"])
        # Eq. 5 overestimates the density at screening (the paper reports a
        # factor 1.5-2; energy balance with Eq. 10 gives a factor 2)
        assert 0.25 < r["n_s"] / r["n_s_eq5"] < 0.7, (r["n_s"], r["n_s_eq5"])
        # section 4, Eq. 10
        assert 0.8 < r["gmean_s"] / r["gmean_eq10"] < 1.7, (r["gmean_s"], r["gmean_eq10"])
        # section 4, Eq. 8: at screening the spectrum is exponential in gamma
        # below gamma_thr, with a slope near ln(2/f) / gamma_thr (shallower
        # as the mean is higher than Eq. 10) and a mean of 1 / slope
        sp = spectrum_fit(cfg, samples, spectra, r["i_s"])
        print("Eq. 8", sp)
        assert sp["r2"] > 0.85, sp
        assert 0.5 < -sp["slope"] / math.log(2.0 / f) < 1.1, sp
        assert 0.8 < sp["mean_gamma"] * -sp["slope"] / gthr < 1.2, sp
    else:
        # One pair per cell screens E0 as the second generation starts to
        # emit: the first generation alone multiplies the seed by about
        # 1 + 2/f, more than screening needs.  No exponential phase exists,
        # so the relations of sections 3-4 that assume one are not checked.
        assert r["t_s"] < 3.0 * r["t_a"] and r["growth_s"] < 1.0 + 2.0 / f, r
    # section 5: four half periods of the oscillation against omega_0
    hp = r["half_periods"]
    assert len(hp) >= 4, hp
    for x in hp[:4]:
        assert abs(x["omega"] / x["omega_th"] - 1.0) < 0.08, x
        if f >= 0.01:
            # <1/gamma^3> of the exponential distribution of Eq. 8 over
            # [1, gamma_thr] is about ln(2/f) / (2 gamma_thr)
            assert 0.8 < x["inv_g3"] / r["inv_g3_exp"] < 2.0, (x, r["inv_g3_exp"])
    if f == 0.1 and precision == workloads.MIXED:
        # section 6: one secondary burst per cycle, peaking in the last tenth
        # or so of a half period, just before <E> returns to zero
        for c in range(4):
            x, y = hp[2 * c], hp[2 * c + 1]
            big, small = (x, y) if x["pairs"] > y["pairs"] else (y, x)
            assert small["pairs"] < 0.2 * big["pairs"], (x, y)
            assert big["burst_at"] > 0.8, big
        # Eq. 24 over three cycles.  The jump conditions of section 6 keep
        # E omega continuous across a burst, so the amplitude falls at least
        # by the measured jump of omega^2; the fitted eps0 lies within a
        # factor 2 of that jump.
        d = damping_fit(hp, 3)
        print(d)
        assert d["amp_loss_per_cycle"] > 0.01, d
        assert 0.8 < d["eps0_fit"] / d["eps_omega"] < 2.0, d


def _window_growth(cfg, h, t_a, width=0.5, start=1.0, stop=4.0):
    """Growth rates of ln N over consecutive windows of `width` t_a."""
    t = (h["step"] + 1) * cfg["dt"]
    lnN = np.log(h["n_minus"].astype(np.float64))
    out = []
    for a in np.arange(start, stop, width):
        sel = (t > a * t_a) & (t < (a + width) * t_a)
        out.append(float(np.polyfit(t[sel], lnN[sel], 1)[0]))
    return np.array(out)


def test_threshold_spread_smooths_the_cascade():
    """A spread of the threshold, which the paper's conclusion names as
    absent from its model and as a possible smoother of the distribution:
    each lepton's own threshold uniform in gamma_thr (1 +/- 0.25), f = 0.1 at
    the section 3 scale, against the same run without it.  The mean delay
    to threshold is unchanged, so the growth still follows Eqs. 1-2 and
    section 5 still gives omega_0; the generations overlap, so the growth
    measured over half-t_a windows swings less; fewer leptons sit at one
    threshold, so the secondary bursts of section 6 damp the oscillation
    less."""
    res = {}
    for spread in (0.0, 0.25):
        cfg, h, samples, _ = run_uniform_cascade(0.1, workloads.MIXED, 500.0, 12000, spread)
        r = measure(cfg, h, samples)
        r["windows"] = _window_growth(cfg, h, r["t_a"])
        r["damping"] = damping_fit(r["half_periods"], 3)
        res[spread] = r
        print(spread, {k: v for k, v in r.items() if k != "half_periods"})
    a, b = res[0.0], res[0.25]
    assert b["energy_drift"] < 2e-3
    assert abs(b["G"] / b["G_exact"] - 1.0) < 0.08, (b["G"], b["G_exact"])
    for x in b["half_periods"][:4]:
        assert abs(x["omega"] / x["omega_th"] - 1.0) < 0.08, x
    assert np.std(b["windows"]) < 0.7 * np.std(a["windows"]), (a["windows"], b["windows"])
    assert b["damping"]["amp_loss_per_cycle"] < 0.7 * a["damping"]["amp_loss_per_cycle"], (
        a["damping"], b["damping"])


def test_nonuniform_gap_screens_on_the_local_clock():
    """The non-uniform start of the paper's conclusion at the section 3
    resolution: E0 exp(-x / (L/4)) from the surface wall and a seed of
    density exp(-x / (L/4)).  Ampere's law is local in 1D and leptons cross
    only a few percent of L before screening, so each altitude screens on
    its own clock: t_s of section 3 with the local E and seed density (the
    growth rate from Eqs. 1-2 at the local t_a).  Measured: the first step
    at which the mean E over a twentieth of the gap turns negative."""
    import torch

    from tests.pic_cases import make_gpu
    cfg = workloads.nonuniform_gap()
    steps, every, nb = 24000, 100, 20
    cfg = dict(cfg, history_rows=steps + 8, diag_every=1)
    g = make_gpu(cfg, stream=torch.cuda.Stream())
    try:
        Es = []
        for _ in range(steps // every):
            g.step_n(every)
            Es.append(g.read_fields(rho=False)["E"])
        h = g.read_history()
    finally:
        g.close()
        del g
        torch.cuda.empty_cache()
    Es = np.array(Es)
    nc, dt, e0, gthr, f = cfg["n_cells"], cfg["dt"], cfg["e0"], cfg["gamma_thr"], cfg["f"]
    L = nc * cfg["dx"]
    W = h["kinetic"] + h["field"] + h["photon_energy"] + h["lost_energy"]
    assert np.max(np.abs(W / W[0] - 1.0)) < 1e-3
    ls = 0.25 * L                      # seed scale height
    npairs = len(cfg["explicit"][0][0])
    rows = []
    for b in range(nb):
        x = (b + 0.5) / nb * L
        Eb = Es[:, b * nc // nb:(b + 1) * nc // nb].mean(axis=1)
        neg = np.nonzero(Eb < 0.0)[0]
        Ex = e0 * math.exp(-x / (0.25 * L))
        n0 = npairs * cfg["weight"] * math.exp(-x / ls) / (ls * -math.expm1(-L / ls))
        ta = A.t_accel(Ex, gthr)
        t_form = A.screening_time(Ex, n0, A.growth_rate_exact(f, ta))
        t_meas = (neg[0] + 1) * every * dt if neg.size else float("nan")
        rows.append((b, t_meas, t_form))
    print(rows)
    screened = [r for r in rows if not math.isnan(r[1])]
    assert len(screened) >= nb // 2, rows
    for b, tm, tf in screened:
        assert 0.9 < tm / tf < 1.3, (b, tm, tf)
    t = [r[1] for r in screened]
    assert all(a < c for a, c in zip(t[:-1], t[1:])), t  # the front moves up


def test_corotating_gap_at_paper_scale():
    """Section 7's co-rotating gap at the paper's scale: L = 1000 c/omega_p,GJ
    in 10000 cells, dt = 1e-3, j_m = -1.5 rho_GJ c, gamma_thr = 5000,
    f = 0.01, pairs in place, to t = 300.  The two-density cold loading is an
    equilibrium, so E stays zero in the bulk (to the rounding of the loaded
    velocities).  A gap opens at the
    wall the positrons leave through, its field growing linearly in time.
    No lepton can gain more than the gap's potential drop, so the first
    pairs appear only once that drop exceeds gamma_thr, and next to that
    wall.  The bursts then screen the gap field."""
    import torch

    from tests.pic_cases import make_gpu
    steps, every = 300000, 1000
    cfg = dict(workloads.corotating_gap(), history_rows=steps // 10 + 8, diag_every=10)
    g = make_gpu(cfg, stream=torch.cuda.Stream())
    try:
        g.set_event_map(500, every, steps // every)
        Es = []
        for _ in range(steps // every):
            g.step_n(every)
            Es.append(g.read_fields(rho=False)["E"])
        emap = g.read_event_map()
        assert g.read_moments().status == 0
    finally:
        g.close()
        del g
        torch.cuda.empty_cache()
    E = np.array(Es)  # row r: E after (r + 1) * every steps, t = r + 1
    nc, dx = cfg["n_cells"], cfg["dx"]
    # the loaded streams' binary32 velocities differ from j_m in the last
    # bits: at most steps * j_m dt * 2^-23 ~ 5e-5 of drift in the bulk
    bulk = E[:, int(0.3 * nc):int(0.7 * nc)]
    assert np.abs(bulk).max() < 1e-4, np.abs(bulk).max()
    rows = np.nonzero(emap.sum(axis=1))[0]
    assert rows.size > 0
    first = int(rows[0])  # pairs first made during t in (first, first + 1]
    emax = np.abs(E).max(axis=1)
    peak_at = np.argmax(np.abs(E), axis=1)
    # before the first pairs the field peaks at the last cells of the right wall
    assert np.all(peak_at[:first] >= nc - 10), peak_at[:first].min()
    # and grows linearly in time
    assert abs(emax[99] / emax[49] - 2.0) < 0.1, (emax[49], emax[99])
    # the potential drop across the gap (the bulk carries none)
    V = E.sum(axis=1) * dx
    gthr = cfg["gamma_thr"]
    assert V[first - 1] >= gthr and V[first] <= 3.0 * gthr, (V[first - 1], V[first])
    # the first pairs are made next to that wall
    assert np.nonzero(emap[first])[0].min() >= int(0.9 * emap.shape[1])
    # the bursts screen the gap field
    assert emax[-1] < 0.6 * emax[first], (emax[first], emax[-1])
    print("first pairs at t", first + 1, "drop", V[first], "E max", emax[first], "->", emax[-1])
