"""Test helpers: build the same seeded gap on the HIP path and in the oracle,
and compare what they produce."""
import numpy as np

import workloads

HIST_INT = ("step", "n_minus", "n_plus", "n_photons", "pairs_created", "photons_emitted",
            "photons_escaped", "absorbed_minus", "absorbed_plus")
HIST_FLOAT = ("kinetic", "field", "photon_energy", "lost_energy")


def gap_kwargs(cfg):
    kw = {k: cfg[k] for k in workloads.GAP_KEYS}
    for k in ("j_m", "gamma_thr_spread", "shape"):
        if cfg.get(k, 0):
            kw[k] = cfg[k]
    return kw


def make_oracle(cfg, capacity=0):
    import oracle
    g = oracle.OracleGap(**gap_kwargs(cfg), capacity=capacity)
    if cfg.get("n_pairs", 0):
        g.seed(cfg.get("seed_mode", workloads.SEED_RANDOM), cfg["n_pairs"],
               cfg.get("macro_per_pair", 1), cfg.get("p0_minus", 0.0), cfg.get("p0_plus", 0.0))
    for sp, (cell, off, p, ids) in sorted(cfg.get("explicit", {}).items()):
        g.seed_explicit(sp, cell, off, p, ids)
    if cfg.get("E_init") is not None:
        g.set_fields(cfg["E_init"])
    return g


def gpu_params(cfg, **over):
    import paper_2012_05587_amd as P
    c = dict(cfg)
    c.update(over)
    return P.make_params(
        c["n_cells"], c["dx"], c["dt"], c["boundary"], c["e0"], c["gamma_thr"], c["f"],
        c["l_gamma"], c["weight"], int(c["capacity"]), int(c.get("photon_capacity", c["capacity"])),
        c["seed"], c["precision"], c.get("sort_every", 0), c.get("diag_every", 0),
        c.get("history_rows", 0), c.get("j_m", 0.0), c.get("gamma_thr_spread", 0.0),
        c.get("shape", 0))


def make_gpu(cfg, stream=None, **over):
    import paper_2012_05587_amd as P
    g = P.Gap(gpu_params(cfg, **over), stream=stream)
    if cfg.get("n_pairs", 0):
        g.seed_particles(cfg.get("seed_mode", workloads.SEED_RANDOM), cfg["n_pairs"],
                         cfg.get("macro_per_pair", 1), cfg.get("p0_minus", 0.0),
                         cfg.get("p0_plus", 0.0))
    for sp, (cell, off, p, ids) in sorted(cfg.get("explicit", {}).items()):
        g.seed_explicit(sp, cell, off, p, ids)
    if cfg.get("E_init") is not None:
        g.set_fields(cfg["E_init"])
    return g


def by_id(P):
    o = np.argsort(P["id"], kind="stable")
    return {k: v[o] for k, v in P.items()}


def compare_history(hg, ho, rtol=1e-9):
    """Integer columns bit-exact; binary64 sums within rtol (summation order)."""
    assert len(hg) == len(ho), (len(hg), len(ho))
    for k in HIST_INT:
        bad = np.nonzero(hg[k] != ho[k])[0]
        assert bad.size == 0, f"{k} differs first at row {bad[0]}: {hg[k][bad[0]]} vs {ho[k][bad[0]]}"
    for k in HIST_FLOAT:
        scale = np.maximum(np.abs(ho[k]), 1e-300)
        err = np.max(np.abs(hg[k] - ho[k]) / scale) if len(ho) else 0.0
        assert err <= rtol, f"{k}: rel err {err}"
    emax = max(np.max(np.abs(ho["e_mean"])) if len(ho) else 0.0, 1e-300)
    assert np.max(np.abs(hg["e_mean"] - ho["e_mean"])) <= rtol * emax if len(ho) else True


def compare_particles(gg, go, ptol):
    """Same ids, same cells and offsets, momenta within ptol * max(|p|, 1)."""
    stats = {}
    for s in (0, 1):
        a = by_id(gg.read_particles(s))
        b = by_id(go.particles(s))
        assert len(a["id"]) == len(b["id"]), (s, len(a["id"]), len(b["id"]))
        assert np.array_equal(a["id"], b["id"])
        assert np.array_equal(a["cell"], b["cell"])
        assert np.array_equal(a["off"], b["off"])
        dp = np.abs(a["p"] - b["p"]) / np.maximum(np.abs(b["p"]), 1.0)
        stats[s] = float(dp.max()) if dp.size else 0.0
        assert stats[s] <= ptol, (s, stats[s])
    return stats


def compare_fields(gg, go, rtol=1e-4):
    Eg = gg.read_fields(rho=False)["E"]
    Eo = go.fields()["E"]
    err = np.max(np.abs(Eg - Eo)) / max(np.max(np.abs(Eo)), 1e-300)
    assert err <= rtol, err
    return err, bool(np.array_equal(Eg, Eo))


def gauss_residual(E, rho, periodic):
    if periodic:
        return (E - np.roll(E, 1)) - rho[:-1]
    return (E[1:] - E[:-1]) - rho[1:-1]
