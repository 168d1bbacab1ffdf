"""GPU tests of the capacity freeze, the emission direction at the energy
boundary, the preparation of a gap, and the order independence of the
binary64 diagnostics (needs a GPU; every case also runs the oracle).

Capacity bounds live leptons on both sides: a gap freezes after the step at
which a species holds more live leptons than the capacity, whatever the
re-sort cadence and however many slots absorbed leptons still hold.
"""
import math

import numpy as np
import pytest

import workloads
from tests import pic_cases as pc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_05587_amd as P
    P.lib()
    yield


@pytest.mark.parametrize("sort_every", [40, 7, 0])
@pytest.mark.parametrize("precision", [workloads.FP64, workloads.MIXED])
def test_live_capacity_freezes_at_the_oracles_step(precision, sort_every):
    """Configuration 1 with 9500 live leptons per species: its absorbing walls
    have removed leptons since the last re-sort when the count first passes
    the capacity, so counting slots would freeze earlier.  GPU and oracle
    freeze at the same step with PIC_ERR_CAPACITY, and the rows before it
    agree."""
    import torch
    import paper_2012_05587_amd as P
    cfg = workloads.config("c1_fp64_reference_gap")
    cfg.update(precision=precision, capacity=9500, history_rows=400)
    print(f"[case] live capacity prec={precision} sort_every={sort_every}", flush=True)
    go = pc.make_oracle(cfg, capacity=9500)
    assert go.step(400) == -3
    ho = go.history()
    n_freeze = go.steps_done
    # leptons were absorbed between the last multiple of 7 and the freeze
    last = (n_freeze // 7) * 7 - 1
    assert ho["absorbed_minus"][-1] > ho["absorbed_minus"][last]
    stream = torch.cuda.Stream() if sort_every != 7 else None
    gg = pc.make_gpu(cfg, stream=stream, sort_every=sort_every)
    rep = gg.step_n(400, report=True)
    assert rep.status == P.ERR_CAPACITY
    assert rep.steps_done == n_freeze
    pc.compare_history(gg.read_history(), ho)
    m = gg.read_moments()
    assert m.n_minus <= 9500 and m.n_plus <= 9500
    with pytest.raises(P.PicError):
        gg.step_n(1)


@pytest.mark.parametrize("precision,p_exact", [(workloads.MIXED, 3.872983455657959),
                                                (workloads.FP64, 3.872983346207417)])
@pytest.mark.parametrize("l_gamma", [0.0, 5.0])
def test_emitter_left_at_rest_keeps_its_direction(precision, p_exact, l_gamma):
    """gamma_thr = 4, f = 3/4: a lepton at gamma = 4 is left at rest by its
    emission.  Its children (or photon) move the way it moved, on the GPU as
    in the oracle, and its stored momentum keeps the sign."""
    cfg = dict(n_cells=32, dx=1.0, dt=0.45, boundary=workloads.PERIODIC, e0=0.0, gamma_thr=4.0,
               f=0.75, l_gamma=l_gamma, weight=0.0, seed=17, precision=precision,
               capacity=1000, photon_capacity=1000, history_rows=16)
    ex = {s: ([5, 9], [0.25, 0.75], [p_exact, -p_exact], [10 + s, 20 + s]) for s in (0, 1)}
    cfg["explicit"] = ex
    go = pc.make_oracle(cfg)
    assert go.step(3) == 0
    gg = pc.make_gpu(cfg)
    gg.step_n(3)
    pc.compare_history(gg.read_history(), go.history())
    for s in (0, 1):
        a, b = pc.by_id(gg.read_particles(s)), pc.by_id(go.particles(s))
        assert np.array_equal(a["id"], b["id"])
        assert np.array_equal(a["cell"], b["cell"]) and np.array_equal(a["off"], b["off"])
        assert np.array_equal(np.signbit(a["p"]), np.signbit(b["p"]))
        assert np.array_equal(a["p"], b["p"])
    if l_gamma > 0:
        pg, po = gg.read_photons(), go.photons()
        key = lambda d: sorted(zip(d["xq"].tolist(), d["conv_step"].tolist(), d["dir"].tolist(),  # noqa: E731
                                   d["child"].tolist()))
        assert key(pg) == key(po)


def test_seeding_a_seeded_gap_is_refused():
    """Seed ids start at 0, so a second random seeding of a gap would repeat
    ids (and with them random streams): refused as in the oracle."""
    import paper_2012_05587_amd as P
    cfg = workloads.config("c1_fp64_reference_gap")
    gg = pc.make_gpu(cfg)
    with pytest.raises(P.PicError) as e:
        gg.seed_particles(workloads.SEED_RANDOM, 4, 1)
    assert e.value.status == P.ERR_STATE
    gg.step_n(2)
    assert gg.read_moments().n_minus == cfg["n_pairs"] * cfg["macro_per_pair"]


@pytest.mark.parametrize("precision", [workloads.FP64, workloads.MIXED])
def test_prepared_gap_matches_unprepared_and_oracle(precision):
    """pic_prepare (seed sorted, graphs captured before the first step) changes
    nothing but when the work happens: the run equals an unprepared one bit for
    bit, history included, and the oracle."""
    import torch
    cfg = workloads.config("c1_fp64_reference_gap")
    cfg.update(precision=precision, history_rows=700)
    out = []
    for prep in (True, False):
        gg = pc.make_gpu(cfg, stream=torch.cuda.Stream())
        if prep:
            gg.prepare()
        gg.step_n(600)
        out.append((gg.read_history(), gg.read_fields(rho=False)["E"], gg))
    for k in out[0][0].dtype.names:
        assert np.array_equal(out[0][0][k], out[1][0][k]), k
    assert np.array_equal(out[0][1], out[1][1])
    go = pc.make_oracle(cfg)
    assert go.step(600) == 0
    pc.compare_history(out[0][0], go.history())
    pc.compare_particles(out[0][2], go, 1e-12 if precision == workloads.FP64 else 1e-5)


def test_prepared_batch_matches_unprepared():
    """A prepared batch of 12 gaps of the batched scan steps bit for bit like
    an unprepared one."""
    import torch
    import paper_2012_05587_amd as P
    gaps = workloads.batched_scan(12, precision=workloads.MIXED, steps=300)
    for c in gaps:
        c.update(capacity=300_000, photon_capacity=600_000, history_rows=400)
    hs = []
    for prep in (True, False):
        b = P.Batch([pc.gpu_params(c) for c in gaps], stream=torch.cuda.Stream())
        for v, c in zip(b.gaps, gaps):
            v.seed_particles(workloads.SEED_RANDOM, c["n_pairs"], c["macro_per_pair"])
        if prep:
            b.prepare()
        b.step_n(300)
        hs.append([v.read_history() for v in b.gaps])
        b.close()
    for ha, hb in zip(*hs):
        for k in ha.dtype.names:
            assert np.array_equal(ha[k], hb[k]), k


@pytest.mark.parametrize("precision", [workloads.FP64, workloads.MIXED])
def test_diagnostics_do_not_depend_on_lepton_order(precision):
    """The binary64 sums of the history (kinetic, field, lost energy, <E>) are
    exact sums of terms rounded once onto a fixed grid, so they come out bit
    for bit the same whatever the order of the leptons: two runs, and runs at
    re-sort cadences 5, 23 and tuned, agree in every column."""
    import torch
    cfg = workloads.config("c1_fp64_reference_gap")
    cfg.update(precision=precision, history_rows=900)
    runs = []
    for se in (0, 0, 5, 23):
        gg = pc.make_gpu(cfg, stream=torch.cuda.Stream(), sort_every=se)
        gg.step_n(800)
        runs.append(gg.read_history())
    for h in runs[1:]:
        for k in runs[0].dtype.names:
            assert np.array_equal(runs[0][k], h[k]), k
    go = pc.make_oracle(cfg)
    assert go.step(800) == 0
    pc.compare_history(runs[0], go.history())
    # the energies are binary64 re-evaluations from the stored momenta
    ho = go.history()
    assert np.max(np.abs(runs[0]["kinetic"] - ho["kinetic"]) / ho["kinetic"]) < 1e-12


@pytest.mark.parametrize("precision", [workloads.FP64, workloads.MIXED])
def test_photon_tail_past_the_key_horizon(precision):
    """Re-sorts 300 steps apart: between steps 255 and 300 after a sort the
    unsorted photons are found by their stored conversion steps instead of
    their one-byte keys.  History and photons in flight stay the oracle's
    across that range and across the sorts."""
    cfg = workloads.config("c1_fp64_reference_gap")
    cfg.update(precision=precision, history_rows=800)
    go = pc.make_oracle(cfg)
    gg = pc.make_gpu(cfg, sort_every=300)
    done = 0
    for n in (250, 10, 40, 5, 295, 50):  # ends of steps 249, 259, 299, 304, 599, 649
        assert go.step(n) == 0
        gg.step_n(n)
        done += n
        a, b = gg.read_photons(), go.photons()
        key = lambda d: np.lexsort((d["child"], d["dir"], d["conv_step"], d["xq"]))  # noqa: E731
        ka, kb = key(a), key(b)
        assert len(ka) == len(kb), (done, len(ka), len(kb))
        for k in ("xq", "conv_step", "dir", "child"):
            assert np.array_equal(np.asarray(a[k])[ka], np.asarray(b[k])[kb]), (done, k)
    h = gg.read_history()
    pc.compare_history(h, go.history())
    # photons converted in the range the keys do not cover
    assert h["pairs_created"][298] > h["pairs_created"][256]
