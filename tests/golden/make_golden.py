"""Writes the stored expected values of tests/golden/ from the oracle alone.

Run from the repository root:  python tests/golden/make_golden.py
It calls only the oracle (oracle/), on the seeded inputs of workloads/, and
never the HIP path.  Files written:

  c5_fp64_oracle_200_steps.txt
      The large mixed-precision configuration's physics (65536 cells,
      E0 = 1000, gamma_thr = 500, l_gamma = 200 cells, 16384 seed pairs) run
      by the binary64 oracle for its first 200 steps: one history row per
      step (counts; kinetic, field, photon and lost energy; <E>).  The GPU's
      mixed-precision run is compared with it for energy conservation.

  c2_fp64_oracle_statistics.txt
      The binary64 single gap (8192 cells, E0 = gamma_thr = 200,
      l_gamma = 50, 1024 seed pairs) run by the oracle for 3000 steps:
      growth rate of N- (section 3), screening step, amplitude and angular
      frequency of the oscillation of <E> (section 5), with the N- and <E>
      series they are computed from.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402
from tests import cascade_stats as cs  # noqa: E402

COLS = ("step", "n_minus", "n_plus", "n_photons", "pairs_created", "photons_emitted",
        "photons_escaped", "absorbed_minus", "absorbed_plus", "kinetic", "field",
        "photon_energy", "lost_energy", "e_mean")


def run(cfg, steps):
    kw = {k: cfg[k] for k in workloads.GAP_KEYS}
    kw["precision"] = oracle.FP64
    g = oracle.OracleGap(**kw, capacity=0)
    g.seed(cfg.get("seed_mode", workloads.SEED_RANDOM), cfg["n_pairs"], cfg["macro_per_pair"])
    t0 = time.time()
    st = g.step(steps)
    print(f"{steps} steps in {time.time() - t0:.0f} s, status {st}", flush=True)
    assert st == oracle.OK
    return g.history()


def write_rows(path, header, rows):
    with open(path, "w") as f:
        for line in header:
            f.write(f"# {line}\n")
        f.write("# " + " ".join(COLS) + "\n")
        for r in rows:
            f.write(" ".join(str(int(r[c])) if r.dtype[c].kind == "i" else repr(float(r[c]))
                             for c in COLS) + "\n")


def c5():
    cfg = workloads.config("c5_large_mixed")
    h = run(cfg, 200)
    write_rows(os.path.join(HERE, "c5_fp64_oracle_200_steps.txt"),
               ["Oracle (binary64) history of the large gap of the benchmark configurations:",
                "65536 cells, dx = 1, dt = 0.45, absorbing, E0 = 1000, gamma_thr = 500, f = 0.5,",
                f"l_gamma = 200 cells, 16384 random seed pairs at rest, seed {cfg['seed']}.",
                "Written by tests/golden/make_golden.py from the oracle alone."], h)


def c2():
    cfg = workloads.config("c2_fp64_single_gap")
    steps = 3000
    h = run(cfg, steps)
    dt = cfg["dt"]
    n0 = cfg["n_pairs"] * cfg["macro_per_pair"]
    rate, a, b = cs.growth_rate(h["n_minus"], dt, n0)
    ts = cs.screening_step(h["e_mean"])
    omega, amp, zs = cs.oscillation(h["e_mean"], dt, ts)
    with open(os.path.join(HERE, "c2_fp64_oracle_statistics.txt"), "w") as f:
        f.write("# Oracle (binary64) run of the single gap of the benchmark configurations:\n")
        f.write("# 8192 cells, dx = 1, dt = 0.45, absorbing, E0 = gamma_thr = 200, f = 0.5,\n")
        f.write(f"# l_gamma = 50 cells, 1024 random seed pairs at rest, seed {cfg['seed']}; {steps} steps.\n")
        f.write("# Statistics of tests/cascade_stats.py; written by tests/golden/make_golden.py.\n")
        f.write(f"growth_rate {rate!r} {a} {b}\n")
        f.write(f"screening_step {ts}\n")
        f.write(f"omega {omega!r}\n")
        f.write(f"amplitude {amp!r}\n")
        f.write("zero_crossings " + " ".join(repr(float(z)) for z in zs) + "\n")
        f.write("n_minus " + " ".join(str(int(x)) for x in h["n_minus"][:ts + 1]) + "\n")
        hi = int(np.ceil(zs[-1])) + 2
        f.write("e_mean " + " ".join(repr(float(x)) for x in h["e_mean"][:hi]) + "\n")
    print(f"growth {rate:.5f} over steps {a}-{b}, screening {ts}, omega {omega:.5f}, amplitude {amp:.4f}")


if __name__ == "__main__":
    which = sys.argv[1:] or ["c5", "c2"]
    for w in which:
        {"c5": c5, "c2": c2}[w]()
