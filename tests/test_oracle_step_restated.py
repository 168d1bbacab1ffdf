"""Pins of the oracle's seeding and of one step's per-operation rounding.

The oracle runs every per-particle operation of the mixed path in binary32
(a binary64 result of +, -, *, / or sqrt of binary32 operands, rounded once)
and of the binary64 path in binary64.  Here one step of many independent
leptons is restated with numpy scalars, whose float32 and float64 arithmetic
rounds every one of those operations correctly, and numpy's own Philox
generator.  The restatement follows the step as the paper's model fixes it
(section 2: emission at gamma_thr, pair energy f gamma_thr split equally,
the emitter keeping its direction; Eq. 4 with the readings of the oracle
for the gather and the fixed-point move), written from that description and
not from the oracle's code.  Zero weight keeps E frozen, so every lepton is
its own case; the fields, offsets and momenta are random, so a dropped
rounding, a swapped operand or a wrong sign in any operation shows up as a
bit difference in some of the thousands of leptons.

The seeding is pinned the same way: random seeding against numpy's Philox
with the seed recipe, plus a chi-square test of uniformity (section 3 seeds a
uniform plasma); lattice seeding against exact rational positions.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle
from tests import brute_tree

TAG_SEED, TAG_PHOTON = 1, 2


# ------------------------------------------------------------------ seeding
def test_random_seed_matches_numpy_philox():
    """Pair i: u = Philox4x64-10(key (i, seed), counter (0, 0, 1, 0)); cell =
    hi32(u0) * N_c >> 32, offset = top 24 bits of u1 times 2^-24; electron id
    2i and positron id 2i + 1 at one point, both at the seeded momenta."""
    nc, npairs, seed = 777, 300, 2012055871
    for prec, K in ((oracle.FP64, 40), (oracle.MIXED, 24)):
        g = oracle.OracleGap(n_cells=nc, dx=1.0, dt=0.45, boundary=oracle.ABSORBING, e0=1.0,
                             gamma_thr=100.0, f=0.5, l_gamma=0.0, weight=1.0, seed=seed,
                             precision=prec)
        g.seed(oracle.SEED_RANDOM, npairs, 1, -0.25, 1.5)
        e, p = g.particles(0), g.particles(1)
        assert len(e["id"]) == len(p["id"]) == npairs
        for i in range(npairs):
            u = brute_tree.philox((0, 0, TAG_SEED, 0), (i, seed))
            cell = ((u[0] >> 32) * nc) >> 32
            off = (u[1] >> 40) / 2.0**24
            assert e["id"][i] == 2 * i and p["id"][i] == 2 * i + 1
            assert e["cell"][i] == cell and p["cell"][i] == cell
            assert e["off"][i] == off and p["off"][i] == off
        assert np.all(e["p"] == -0.25) and np.all(p["p"] == 1.5)
        # a second seeding of the same gap is refused, as on the device
        with pytest.raises(RuntimeError):
            g.seed(oracle.SEED_RANDOM, 1, 1)


def test_random_seed_is_uniform():
    """Cells and offsets of a random seed pass a chi-square test of uniformity
    (section 3 seeds a uniform pair plasma)."""
    nc, npairs = 64, 40_000
    g = oracle.OracleGap(n_cells=nc, dx=1.0, dt=0.45, boundary=oracle.PERIODIC, e0=1.0,
                         gamma_thr=100.0, f=0.5, l_gamma=0.0, weight=1.0, seed=99)
    g.seed(oracle.SEED_RANDOM, npairs, 1)
    e = g.particles(0)
    counts = np.bincount(e["cell"], minlength=nc)
    assert stats.chisquare(counts).pvalue > 1e-4
    ob = np.bincount(np.floor(e["off"] * 50).astype(int), minlength=50)
    assert stats.chisquare(ob).pvalue > 1e-4
    # the position along the gap, x = cell + offset, is uniform too
    x = e["cell"] + e["off"]
    assert stats.kstest(x / nc, "uniform").pvalue > 1e-4


@pytest.mark.parametrize("nc,npairs", [(512, 1024), (1000, 333), (7, 10), (64, 64)])
def test_lattice_seed_is_evenly_spaced(nc, npairs):
    """Lattice seeding puts pair i at x_i = (i + 1/2) N_c / N, on the 2^-24
    grid below it (exact rational arithmetic; the binary64 evaluation may
    differ by one grid unit only where x_i lies within rounding of a grid
    point)."""
    g = oracle.OracleGap(n_cells=nc, dx=1.0, dt=0.45, boundary=oracle.PERIODIC, e0=1.0,
                         gamma_thr=100.0, f=0.5, l_gamma=0.0, weight=1.0, seed=5)
    g.seed(oracle.SEED_LATTICE, npairs, 1)
    for s in (0, 1):
        P = g.particles(s)
        X = P["cell"].astype(np.int64) * 2**24 + np.rint(P["off"] * 2**24).astype(np.int64)
        for i in range(npairs):
            exact = Fraction(2 * i + 1, 2) * Fraction(nc, npairs) * 2**24
            fl = math.floor(exact)
            if X[i] != fl:
                assert X[i] == fl - 1 and exact - fl < Fraction(1, 2**20), (i, X[i], exact)
        assert np.all(np.diff(X) > 0)


# --------------------------------------------------- one step, restated
def _node_e(E, c, periodic):
    """E at cell centre c as the gather sees it: wrapped, or the edge value
    repeated beyond an absorbing wall."""
    n = len(E)
    if periodic:
        return E[c % n]
    return E[min(max(c, 0), n - 1)]


def _spline(X, K):
    """Nearest node j = floor(X 2^-K + 1/2) and the integer weights of the
    nodes j-1, j, j+1: (1/2 - d)^2/2 and (1/2 + d)^2/2 rounded down, the
    middle one the rest of 2^K (X in units of 2^-K cells from node 0)."""
    one, half = 1 << K, 1 << (K - 1)
    j = (X + half) // one
    d = X - j * one
    wl = ((half - d) ** 2) >> (K + 1)
    wr = ((half + d) ** 2) >> (K + 1)
    return j, (wl, one - wl - wr, wr)


def _restated_step(F, prm, E, leptons, step):
    """One step of independent leptons (zero weight) in frozen E.

    F is the float type (np.float32 or np.float64); leptons is a list of
    (species, cell, offq, p, id).  Returns (survivors {id: (cell, offq, p)},
    children {id: (species, cell, offq, p)}, photons [(xq, conv_step, dir,
    child)], absorbed ids)."""
    K = 24 if F is np.float32 else 40
    one = 1 << K
    nc = prm["n_cells"]
    periodic = prm["boundary"] == oracle.PERIODIC
    dtdx = F(prm["dt"] / prm["dx"])
    thr = F(prm["gamma_thr"])
    gpair = F(prm["f"] * prm["gamma_thr"])
    ghalf = gpair * F(0.5)
    pchild = np.sqrt(ghalf * ghalf - F(1))
    half = F(0.5)
    table = brute_tree.conv_table(prm["dt"], prm["dx"], prm["l_gamma"]) if prm["l_gamma"] > 0 else []
    photon_step = round(prm["dt"] / prm["dx"] * 2**K)  # binary64 product, rounded to the grid
    domain = nc * one
    surv, kids, photons, gone = {}, {}, [], []
    for s, c, oq, p0, pid in leptons:
        q = -1.0 if s == 0 else 1.0
        o = F(oq / one)  # exact: the offset is a multiple of 2^-K
        # gather: node averages of E, interpolated (linear) or spline-weighted
        if prm["shape"] == oracle.SHAPE_LINEAR:
            em, ec, ep = (F(_node_e(E, c + k, periodic)) for k in (-1, 0, 1))
            el = half * (em + ec)
            er = half * (ec + ep)
            ex = el + o * (er - el)
        else:
            j, w = _spline(oq, K)
            e4 = [F(_node_e(E, c + j - 2 + k, periodic)) for k in range(4)]
            en = [half * (e4[k] + e4[k + 1]) for k in range(3)]
            sw = [F(wk) / F(one) for wk in w]
            ex = (sw[0] * en[0] + sw[1] * en[1]) + sw[2] * en[2]
        # push, Lorentz factor, velocity
        p = F(p0) + F(q * prm["dt"]) * ex
        gam = np.sqrt(F(1) + p * p)
        v = p / gam
        dq = int(np.rint(np.float64(v * dtdx) * 2.0**K))
        # move on the fixed-point grid; crossing at most one node
        nq, c2, keep = oq + dq, c, True
        if prm["shape"] == oracle.SHAPE_LINEAR:
            if nq >= one:
                nq -= one
                c2 = c + 1
            elif nq < 0:
                nq += one
                c2 = c - 1
            if c2 < 0 or c2 >= nc:
                if periodic:
                    c2 %= nc
                else:
                    keep = False
        else:
            X = c * one + nq
            if not periodic and (X < 0 or X >= domain):
                keep = False
            else:
                X %= domain
                c2, nq = X // one, X % one
        if not keep:
            gone.append(pid)
            continue
        # emission: gamma_pair per emission while at or above the threshold
        k, gm = 0, gam
        while gm >= thr:
            gm = gm - gpair
            k += 1
        d = 1 if p > 0 else -1
        if k:
            mag = np.sqrt(gm * gm - F(1))
            p = mag if d > 0 else -mag
        surv[pid] = (c2, nq, float(p))
        for jj in range(k):
            bits, u32 = brute_tree.draw_run(pid, prm["seed"], step, jj, TAG_PHOTON)
            child = bits & ~1
            if not table:
                pc = float(pchild if d > 0 else -pchild)
                kids[child] = (0, c2, nq, pc)
                kids[child | 1] = (1, c2, nq, pc)
                continue
            ncv = next(kk for kk in range(1, len(table)) if u32 >= table[kk])
            Xc = c2 * one + nq + d * ncv * photon_step
            if not periodic and (Xc < 0 or Xc >= domain):
                continue  # escapes
            photons.append((Xc % domain, step + ncv, d, child))
    return surv, kids, photons, gone


def _random_case(rng, K, nc, n):
    """n leptons with random cells, grid offsets, momenta (some far above the
    threshold, so that one step emits several times) and ids."""
    cells = rng.integers(0, nc, n)
    offq = rng.integers(0, 1 << K, n)
    # edge cells often, so that leptons leave through the walls
    edge = rng.random(n) < 0.15
    cells[edge] = rng.choice([0, nc - 1], edge.sum())
    mag = np.where(rng.random(n) < 0.5, rng.uniform(0, 3, n), rng.uniform(60, 600, n))
    p = mag * rng.choice([-1.0, 1.0], n)
    ids = rng.choice(2**62, n, replace=False).astype(np.uint64) * 2
    sp = rng.integers(0, 2, n)
    return cells, offq, p, ids, sp


@pytest.mark.parametrize("precision", [oracle.MIXED, oracle.FP64])
@pytest.mark.parametrize("shape", [oracle.SHAPE_LINEAR, oracle.SHAPE_QUADRATIC])
@pytest.mark.parametrize("boundary,l_gamma", [(oracle.ABSORBING, 12.0), (oracle.PERIODIC, 12.0),
                                              (oracle.ABSORBING, 0.0)])
def test_one_step_matches_restatement(precision, shape, boundary, l_gamma):
    """1500 leptons per case, one step in a random frozen field: every
    survivor's cell, offset and momentum, every child and every photon agree
    bit for bit with the numpy restatement."""
    F = np.float32 if precision == oracle.MIXED else np.float64
    K = 24 if precision == oracle.MIXED else 40
    rng = np.random.default_rng(1000 * precision + 10 * shape + boundary + int(l_gamma))
    nc, n, step0 = 40, 1500, 0
    prm = dict(n_cells=nc, dx=1.0, dt=0.45, boundary=boundary, e0=0.0, gamma_thr=100.0, f=0.3,
               l_gamma=l_gamma, weight=0.0, seed=2012055872, precision=precision, shape=shape)
    E = rng.normal(0.0, 40.0, nc)
    cells, offq, p, ids, sp = _random_case(rng, K, nc, n)
    if precision == oracle.MIXED:
        p = p.astype(np.float32).astype(np.float64)
    g = oracle.OracleGap(**prm)
    g.set_fields(E)
    for s in (0, 1):
        m = sp == s
        g.seed_explicit(s, cells[m], offq[m] / 2.0**K, p[m], ids[m] | np.uint64(s))
    assert g.step(1) == oracle.OK
    leptons = [(int(s), int(c), int(o), float(pp), int(i) | int(s))
               for s, c, o, pp, i in zip(sp, cells, offq, p, ids)]
    surv, kids, photons, gone = _restated_step(F, prm, E, leptons, step0)
    # the restated step emits several times per lepton and, with walls, absorbs some
    assert len(gone) > 20 if boundary == oracle.ABSORBING else not gone
    assert len(kids) > 500 or len(photons) > 250
    got = {}
    for s in (0, 1):
        P = g.particles(s)
        for c, o, pp, i in zip(P["cell"], P["off"], P["p"], P["id"]):
            got[int(i)] = (s, int(c), int(round(o * 2**K)), float(pp))
    for pid, (c2, nq, pv) in surv.items():
        s, c, o, pp = got.pop(pid)
        assert (c, o, pp) == (c2, nq, pv), pid
    for cid, val in kids.items():
        assert got.pop(cid) == val, cid
    assert not got  # nothing else survived or was born
    ph = g.photons()
    mine = sorted(zip(ph["xq"].tolist(), ph["conv_step"].tolist(), ph["dir"].tolist(),
                      ph["child"].tolist()))
    assert mine == sorted(photons)
    h = g.history()
    assert h["absorbed_minus"][-1] + h["absorbed_plus"][-1] == len(gone)


def test_energy_diagnostics_are_binary64_in_mixed_precision():
    """North star: energy diagnostics stay binary64.  In mixed precision the
    kinetic energy of the history is the binary64 sum of sqrt(1 + p^2) over the
    stored (binary32) momenta, evaluated in binary64, not the binary32 gamma
    of the push."""
    prm = dict(n_cells=64, dx=1.0, dt=0.45, boundary=oracle.PERIODIC, e0=7.0, gamma_thr=1e300,
               f=0.5, l_gamma=0.0, weight=0.75, seed=3, precision=oracle.MIXED)
    g = oracle.OracleGap(**prm)
    g.seed(oracle.SEED_RANDOM, 500, 1, -3.3, 2.9)
    assert g.step(3) == oracle.OK
    ke = 0.0
    for s in (0, 1):
        for pv in g.particles(s)["p"]:
            ke += 0.75 * math.sqrt(1.0 + pv * pv)
    h = g.history()
    assert abs(h["kinetic"][-1] - ke) <= 1e-13 * ke
    # the binary32 Lorentz factors sum to something measurably different
    ke32 = sum(0.75 * float(np.sqrt(np.float32(1) + np.float32(pv) * np.float32(pv)))
               for s in (0, 1) for pv in g.particles(s)["p"])
    assert abs(ke32 - ke) > 1e-11 * ke


@pytest.mark.parametrize("precision,p_exact", [(oracle.MIXED, 3.872983455657959),
                                                (oracle.FP64, 3.872983346207417)])
@pytest.mark.parametrize("l_gamma", [0.0, 5.0])
def test_emitter_left_at_rest_keeps_its_direction(precision, p_exact, l_gamma):
    """(1 - f) gamma_thr = 1 exactly (gamma_thr = 4, f = 3/4): a lepton at
    gamma = 4 emits once and is left with gamma = 1, |p| = 0.  Its pair (or
    photon) still moves along the direction it had (section 2: the pair
    energy leaves in the emitter's direction), and the emitter's stored
    momentum keeps that sign (+0 or -0)."""
    prm = dict(n_cells=32, dx=1.0, dt=0.45, boundary=oracle.PERIODIC, e0=0.0, gamma_thr=4.0,
               f=0.75, l_gamma=l_gamma, weight=0.0, seed=17, precision=precision)
    g = oracle.OracleGap(**prm)
    for s in (0, 1):
        g.seed_explicit(s, [5, 9], [0.25, 0.75], [p_exact, -p_exact], [10 + s, 20 + s])
    assert g.step(1) == oracle.OK
    for s in (0, 1):
        P = g.particles(s)
        for i, want in ((10 + s, 1.0), (20 + s, -1.0)):
            k = int(np.nonzero(P["id"] == i)[0][0])
            assert P["p"][k] == 0.0 and math.copysign(1.0, P["p"][k]) == want
    if l_gamma == 0.0:
        kids = [g.particles(s) for s in (0, 1)]
        moving = np.concatenate([k["p"][~np.isin(k["id"], [10, 11, 20, 21])] for k in kids])
        cells = np.concatenate([k["cell"][~np.isin(k["id"], [10, 11, 20, 21])] for k in kids])
        assert len(moving) == 8
        # children at the emitter's cell, moving the emitter's way
        assert np.all(moving[cells == 5] > 0) and np.all(moving[cells == 9] < 0)
    else:
        ph = g.photons()
        assert len(ph["dir"]) == 4
        start = ph["xq"] - ph["dir"] * (ph["conv_step"] - 0) * round(0.45 * 2**g.offset_bits)
        assert sorted(ph["dir"].tolist()) == [-1, -1, 1, 1]
        # each photon started at its emitter's position
        cell0 = (start // 2**g.offset_bits) % 32
        assert np.all((cell0 == 5) == (ph["dir"] == 1))
