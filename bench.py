"""Benchmark of the MI355X pair-cascade PIC path: particle-pushes per second.

A step is one PIC time step of the whole path (gather and push, move and
current deposit, Ampere update, emission, conversion, periodic re-sort) for
every lepton of every gap.  A push is one lepton advanced one step, counted
exactly by the device.  Inputs are resident in HBM before timing starts.

Default workload ("mixed-batched vs plain FP64"): 256 independent gaps with
N_cells log-uniform in [1024, 16384], E0 and gamma_thr uniform in [50, 400],
l_gamma uniform in [10, 100] cells and 256-4096 seed pairs, advanced together
for 2000 steps in mixed precision (value).  Beside it: the same batch in
binary64, and the binary64 single gap of 8192 cells (E0 = gamma_thr = 200,
l_gamma = 50, 1024 seed pairs) over its numerically stable first 10000 steps.

Prints one JSON line.  The roofline entry is for the push kernel, which
moves the lepton state: 4 B cell + 4 B offset + 4 B momentum read and written
(24 B per push) in mixed precision, 40 B per push in binary64.  Its time is
summed from HIP events bracketing every push launch on the library's stream,
in a second run of the same steps launched directly (an autotuned re-sort
cadence is tuned there the same way).  The cpu_baseline entry times the
oracle on a bounded sample of the same workload, one gap per process.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0
BYTES_PER_PUSH = {workloads.FP64: 40, workloads.MIXED: 24}
# In steps small enough for it, the push kernel also emits: a stored photon
# writes x 8 + conversion step 4 + child 8 + tail key 1 bytes; an in-place
# pair writes two leptons (cell 4 + offset + momentum + id 8 each).
BYTES_PER_PHOTON = 21
BYTES_PER_CHILD = {workloads.FP64: 28, workloads.MIXED: 20}


def push_alg_bytes(views, gaps, precision):
    """Algorithmic bytes the push kernel moved over a run of these gaps:
    24 (40) B per push, plus the writes of the emissions it drew itself (in
    steps small enough for it to emit; the emitters' id reads are not
    counted)."""
    total = 0
    for v, c in zip(views, gaps):
        m = v.read_moments()
        per = BYTES_PER_PHOTON if c["l_gamma"] > 0 else 2 * BYTES_PER_CHILD[precision]
        total += BYTES_PER_PUSH[precision] * int(m.pushes) + per * int(m.push_emissions)
    return total
DTYPE = {workloads.FP64: "f64", workloads.MIXED: "f32/f64"}
METRIC = "particle-pushes/sec + % HBM roofline, mixed-batched vs plain FP64, 1 MI355X"
# Timed steps when --steps is not given.  The single gap of 8192 cells at
# dt = 0.45 has a non-relativistic omega_p dt far above the leapfrog limit of
# 2 once its plasma cools; after ~10600 steps its field and photon counts grow
# exponentially (a numerical instability the oracle shows identically), so its
# stable first 10000 steps are the job.
DEFAULT_STEPS = {"c2_fp64_single_gap": 10000, "c5_large_mixed": 500, "n1_corotating": 300000}
# The large gap of 65536 cells (E0 = 1000, 16384 seed pairs) screens within
# ~100 steps; its dense plasma is then far from resolved by dt = 0.45 and the
# scheme heats it (total energy +5% by step 500, +12% by step 600, then a
# runaway of photons), so its first 500 steps are the job.  The co-rotating
# gap (10000 cells, dt = 1e-3) opens gaps at its walls whose potential drop
# grows roughly as t^2 / 8; leptons reach gamma_thr = 5000 near t = 200, so
# its job is 300000 steps (t = 300).


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _params(P, c):
    return P.make_params(c["n_cells"], c["dx"], c["dt"], c["boundary"], c["e0"], c["gamma_thr"],
                         c["f"], c["l_gamma"], c["weight"], int(c["capacity"]),
                         int(c["photon_capacity"]), c["seed"], c["precision"],
                         c.get("sort_every", 0), c.get("diag_every", 0), c.get("history_rows", 0),
                         c.get("j_m", 0.0), c.get("gamma_thr_spread", 0.0), c.get("shape", 0))


def _workload(name, precision=None):
    """List of gap configurations of a workload (one for single gaps)."""
    if name == "c4_batched":
        gaps = workloads.batched_scan(256, precision=workloads.MIXED if precision is None else precision)
    elif name == "n1_corotating":
        gaps = [workloads.corotating_gap(precision=workloads.MIXED if precision is None else precision)]
    elif name in ("n3_uniform", "n4_spread", "n4_spline"):
        gaps = [workloads.uniform_cascade(
            0.1, precision=workloads.MIXED if precision is None else precision,
            gamma_thr_spread=0.25 if name == "n4_spread" else 0.0,
            shape=1 if name == "n4_spline" else 0)]
    elif name == "ubench_lattice":
        gaps = [workloads.stream_lattice(precision=workloads.MIXED if precision is None else precision)]
    elif name == "n4_nonuniform":
        gaps = [workloads.nonuniform_gap(precision=workloads.MIXED if precision is None else precision)]
    else:
        gaps = [workloads.config(name)]
        if precision is not None:
            gaps[0]["precision"] = precision
    return gaps


def _make(P, gaps, stream, workspace=None):
    """A Batch of the gaps (or a Gap for one), seeded; `workspace` (a device
    tensor from an earlier batch of the same workload) is reused."""
    if len(gaps) == 1:
        g = P.Gap(_params(P, gaps[0]), stream=stream, workspace=workspace)
        views = [g]
    else:
        g = P.Batch([_params(P, c) for c in gaps], stream=stream, workspace=workspace)
        views = g.gaps
    for v, c in zip(views, gaps):
        if c["n_pairs"]:
            v.seed_particles(c.get("seed_mode", workloads.SEED_RANDOM), c["n_pairs"],
                             c["macro_per_pair"])
        for sp, (cell, off, p, ids) in sorted(c.get("explicit", {}).items()):
            v.seed_explicit(sp, cell, off, p, ids)
        if c.get("E_init") is not None:
            v.set_fields(c["E_init"])
    return g, views


def _frozen(views):
    """Gaps that stopped early: (index, status, steps completed)."""
    out = []
    for i, v in enumerate(views):
        m = v.read_moments()
        if m.status != 0:
            out.append((i, int(m.status), int(m.steps_done)))
    return out


def run_gpu(gaps, steps, warmup=0, reps=5, profile=True, dump=None):
    """Times `steps` steps from the seeded start, `reps` times on fresh
    batches of the same workload (one device workspace, re-created and
    re-seeded to the identical state; graph replay on a side stream), and
    keeps the median.  Before each timed run the batch is prepared (seed
    sorted by cell, step graphs captured and uploaded); that time is reported
    apart.  `warmup` steps of a throwaway batch of the same workload come
    first.  With profile, a further fresh batch runs the same steps launching
    every kernel directly, the push kernel bracketed by HIP events, for that
    kernel's time."""
    import torch
    import paper_2012_05587_amd as P
    P.lib()
    gaps = [dict(c, history_rows=steps + 8) for c in gaps]
    stream = torch.cuda.Stream()
    ws = None
    if warmup > 0:
        g, _ = _make(P, gaps, stream)
        ws = g.workspace
        g.prepare()
        log(f"warm-up: {warmup} steps of the same workload")
        g.step_n(warmup)
        torch.cuda.synchronize()
        g.close()
    runs = []
    for r in range(reps):
        g, views = _make(P, gaps, stream, ws)
        ws = g.workspace
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.prepare()
        t_prep = time.perf_counter() - t0
        log(f"run {r + 1}/{reps}: {steps} steps of {len(gaps)} gap(s), precision {gaps[0]['precision']}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step_n(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pushes = sum(int(v.read_moments().pushes) for v in views)
        done = max(int(v.read_moments().steps_done) for v in views)
        log(f"done in {t1 - t0:.4f} s ({pushes / (t1 - t0):.3e} pushes/s; prepare {t_prep:.3f} s)")
        runs.append(dict(seconds=t1 - t0, prepare_s=t_prep, pushes=pushes, steps=done))
        if r < reps - 1:
            g.close()
    order = sorted(range(reps), key=lambda k: runs[k]["seconds"])
    med = runs[order[reps // 2]]
    peak = 0
    if len(views) == 1:
        h = views[0].read_history()
        peak = int((h["n_minus"] + h["n_plus"]).max()) if len(h) else 0
        if dump:
            import numpy as np
            np.save(dump, h)
    elif dump:
        # per step, summed over the gaps still running: live leptons, photons
        # in flight, cumulative pairs and photons
        import numpy as np
        cols = ("live", "n_photons", "pairs_created", "photons_emitted", "running")
        out_h = np.zeros(steps, dtype=[(c, np.int64) for c in cols])
        for v in views:
            h = v.read_history()
            k = h["step"]
            out_h["live"][k] += h["n_minus"] + h["n_plus"]
            out_h["n_photons"][k] += h["n_photons"]
            # per-step increments of the cumulative counts
            out_h["pairs_created"][k] += np.diff(h["pairs_created"], prepend=0)
            out_h["photons_emitted"][k] += np.diff(h["photons_emitted"], prepend=0)
            out_h["running"][k] += 1
        np.save(dump, out_h)
    tune = g.tuning()
    frozen = _frozen(views)
    out = dict(seconds=med["seconds"], pushes=med["pushes"], steps=med["steps"],
               frozen=len(frozen), frozen_gaps=frozen, peak_leptons=peak,
               prepare_s=[round(x["prepare_s"], 4) for x in runs],
               run_seconds=[round(x["seconds"], 6) for x in runs],
               push_ms=None, push_launches=None, tuning=tune)
    g.close()
    del g, views
    if profile:
        # the evented run launches every kernel directly; an autotuned cadence
        # is tuned there the same way, from the timed S-step segments
        g, views = _make(P, gaps, stream, ws)
        g.profile_push(True)
        log("timing the push kernel with events")
        g.step_n(steps)
        push_ms, launches = g.read_push_time()
        # the evented run repeats the same steps and pushes the same leptons
        again = sum(int(x.read_moments().pushes) for x in views)
        out.update(push_ms=push_ms, push_launches=launches, evented_pushes=again,
                   evented_bytes=push_alg_bytes(views, gaps, gaps[0]["precision"]),
                   evented_photons=sum(int(x.read_moments().push_emissions) for x in views),
                   evented_tuning=g.tuning())
        g.close()
        del g, views
    del ws
    torch.cuda.empty_cache()
    return out


def run_counter_pass(gaps, steps):
    """A bounded run for hardware-counter passes: the workload's first
    `steps` steps launched directly (no graphs), one step at a time, printing
    a line after each, so that a profiler serialising every dispatch still
    shows progress.  Prints a JSON line with the leptons pushed and the push
    kernel's algorithmic bytes per step."""
    import torch
    import paper_2012_05587_amd as P
    P.lib()
    gaps = [dict(c, history_rows=steps + 8) for c in gaps]
    g, views = _make(P, gaps, None)
    g.prepare()
    torch.cuda.synchronize()
    per_step, bytes_step = [], []
    prec = gaps[0]["precision"]
    for k in range(steps):
        before = sum(int(v.read_moments().pushes) for v in views)
        b0 = push_alg_bytes(views, gaps, prec)
        g.step_n(1)
        torch.cuda.synchronize()
        after = sum(int(v.read_moments().pushes) for v in views)
        per_step.append(after - before)
        bytes_step.append(push_alg_bytes(views, gaps, prec) - b0)
        print(f"[pmc] step {k + 1}/{steps}: {after - before} leptons pushed", flush=True)
    print(json.dumps({"counter_pass": True, "steps": steps, "pushes_per_step": per_step,
                      "alg_bytes_per_step": bytes_step}), flush=True)
    g.close()


def measure_copy_gbs(nbytes=1 << 30, reps=10):
    """Bandwidth of a plain device copy (bytes read plus bytes written per
    second, the fastest of `reps` copies of `nbytes`): the streaming ceiling
    the push kernel is also compared with.  Untimed by the benchmark."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / min(times) / 1e9


def _oracle_gap(args):
    c, steps = args
    sys.path.insert(0, ROOT)
    import oracle
    kw = {k: c[k] for k in workloads.GAP_KEYS}
    for k in ("j_m", "gamma_thr_spread", "shape"):
        if c.get(k):
            kw[k] = c[k]
    o = oracle.OracleGap(**kw, capacity=0)
    if c["n_pairs"]:
        o.seed(c.get("seed_mode", workloads.SEED_RANDOM), c["n_pairs"], c["macro_per_pair"])
    for sp, (cell, off, p, ids) in sorted(c.get("explicit", {}).items()):
        o.seed_explicit(sp, cell, off, p, ids)
    if c.get("E_init") is not None:
        o.set_fields(c["E_init"])
    n0 = o.count(0) + o.count(1)
    o.step(steps)
    h = o.history()
    live = (h["n_minus"] + h["n_plus"]).astype("int64")
    return int(n0 + (live[:-1].sum() if len(live) else 0))


def run_cpu_baseline(gaps, steps, procs):
    """The oracle on a bounded sample: the first `steps` steps of each gap,
    one gap per process; pushes per second of wall time."""
    import multiprocessing as mp
    jobs = [(c, steps) for c in gaps]
    log(f"oracle baseline: {len(jobs)} gap(s) x {steps} steps on {procs} process(es)")
    t0 = time.perf_counter()
    if procs > 1:
        with mp.get_context("fork").Pool(procs) as pool:
            pushes = sum(pool.map(_oracle_gap, jobs, chunksize=1))
    else:
        pushes = sum(_oracle_gap(j) for j in jobs)
    t1 = time.perf_counter()
    return dict(value=pushes / (t1 - t0), seconds=t1 - t0, pushes=pushes)


# ----------------------------------------------------------- profiles
PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ("paper_2012_05587_amd/csrc/pic_kernels.hip",
                  "paper_2012_05587_amd/csrc/pic_device.hpp",
                  "paper_2012_05587_amd/csrc/pic_kernels.hpp")


def kernel_source_hash():
    """sha256 over the kernel sources: a stored counter figure is only used
    while the kernels it was taken from are unchanged."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _profile_name(workload, precision):
    return f"k_push_{workload}_{'mixed' if precision == workloads.MIXED else 'fp64'}"


def stored_traffic(workload, precision, steps):
    """HBM bytes per push launch from the committed counter summary of this
    workload and step count, or None when it is missing or the kernel
    sources changed since the counters were taken."""
    path = os.path.join(PROFILE_DIR, _profile_name(workload, precision) + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        prof = json.load(f)
    pmc = prof.get("pmc", {})
    if (prof.get("source_sha256") != kernel_source_hash() or prof.get("workload") != workload
            or pmc.get("steps") != steps or not pmc.get("traffic_bytes_per_launch")):
        return None
    return pmc


def _csv_rows(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def _col(row, *names):
    low = {k.lower(): k for k in row}
    for n in names:
        if n.lower() in low:
            return row[low[n.lower()]]
    raise KeyError(names)


def _counter_per_dispatch(path, counter, match):
    """Per-dispatch values (summed over instances) of `counter` for kernels
    whose name contains `match`, in dispatch order."""
    acc = {}
    for r in _csv_rows(path):
        if _col(r, "Counter_Name") != counter or match not in _col(r, "Kernel_Name"):
            continue
        d = int(_col(r, "Dispatch_Id"))
        acc[d] = acc.get(d, 0.0) + float(_col(r, "Counter_Value"))
    return [acc[d] for d in sorted(acc)]


def summarize(args):
    """Writes profiles/<kernel>_<workload>.{md,json} from rocprofv3 CSV output:
    the kernel trace and stats of the benchmark command (with its printed
    JSON line), and, when given, counter passes (FETCH_SIZE, WRITE_SIZE, the
    LDS counters) over the bounded counter-pass run of the same workload and
    steps, calibrated by the same counters over 1 GiB device copies."""
    import numpy as np
    with open(args.bench_json) as f:
        bench = json.loads([ln for ln in f.read().splitlines() if ln.startswith("{")][-1])
    workload = bench["config"]["workload"]
    prec = workloads.MIXED if bench["dtype"] != "f64" else workloads.FP64
    kname = ("k_push<float, false, false>" if prec == workloads.MIXED
             else "k_push<double, false, false>")
    trace = _csv_rows(args.trace_csv)
    per = {}
    push = []
    for r in trace:
        name = _col(r, "Kernel_Name")
        d = (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) / 1e3
        per.setdefault(name.split("(")[0], []).append(d)
        if kname in name:
            push.append(d)
    # the command's push dispatches in order: the warm-up, `reps` timed runs
    # and the evented run, each of `steps` steps (the warm-up of `warmup`)
    reps = bench["config"].get("timed_runs", {}).get("reps", 1)
    nstep, nwarm = bench["steps"], bench["warmup"]
    timed = push[nwarm:nwarm + reps * nstep]
    evented = push[nwarm + reps * nstep:nwarm + (reps + 1) * nstep]
    total = sum(sum(v) for v in per.values())
    table = sorted(((k, len(v), float(np.mean(v)), sum(v) / 1e3, 100 * sum(v) / total)
                    for k, v in per.items()), key=lambda r: -r[3])
    ev_avg_us = bench["roofline"]["kernel_ms"] * 1e3 / bench["roofline"]["launches"]
    alg = bench["roofline"]["alg_bytes_per_launch"]
    prof = {"kernel": kname, "workload": workload, "steps": bench["steps"],
            "source_sha256": kernel_source_hash(), "commands": args.command, "notes": args.note,
            "trace": {"dispatches": len(push), "avg_us": float(np.mean(push)),
                      "timed_runs_avg_us": float(np.mean(timed)) if timed else None,
                      "evented_run_avg_us": float(np.mean(evented)) if evented else None,
                      "bench_event_avg_us": ev_avg_us,
                      "kernels": [dict(name=k, n=c, mean_us=m, total_ms=t, pct=p)
                                  for k, c, m, t, p in table]},
            "bench": {k: bench[k] for k in ("value", "ms_per_step", "steps")},
            "pmc": {}}
    lines = [f"# {kname} on {workload} ({bench['steps']} timed steps)", "",
             "Commands (from the repository root; rocprofv3 after `cd /tmp && export TMPDIR=/tmp`,",
             "with the repository path for `$R`):", ""]
    lines += [f"    {c}" for c in args.command]
    lines += ["", f"Kernel sources sha256: `{prof['source_sha256']}`", "",
              f"## Kernel trace ({len(push)} dispatches of {kname} in the command)", "",
              f"- rocprofv3 average duration of {kname}, all {len(push)} dispatches: "
              f"{prof['trace']['avg_us']:.2f} us",
              f"- rocprofv3 average over the {len(timed)} dispatches of the {reps} timed runs: "
              f"{np.mean(timed):.2f} us; over the {len(evented)} of the evented run: {np.mean(evented):.2f} us",
              f"- the bench's dispatch-event average over its evented run (the roofline's time): "
              f"{ev_avg_us:.2f} us ({100 * (ev_avg_us / np.mean(evented) - 1):+.1f}% against rocprofv3 "
              "on the same dispatches)", "",
              f"Benchmark line of the same command: {bench['value']:.4g} pushes/s, "
              f"{bench['ms_per_step']:.4f} ms per step, roofline frac {bench['roofline']['frac']:.4f}.", "",
              "| kernel | dispatches | mean us | total ms | % |", "|---|---|---|---|---|"]
    lines += [f"| {k} | {c} | {m:.2f} | {t:.2f} | {p:.1f} |" for k, c, m, t, p in table[:20]]
    if args.fetch_csv and args.write_csv and args.copy_fetch_csv and args.copy_write_csv:
        with open(args.pmc_json) as f:
            cp = json.loads([ln for ln in f.read().splitlines() if ln.startswith("{")][-1])
        pushes = np.array(cp["pushes_per_step"], dtype=float)
        bpp = BYTES_PER_PUSH[prec]

        def factor(path, counter):
            v = [x for x in _counter_per_dispatch(path, counter, "copyBuffer") if x > 0.25 * (1 << 20)]
            return (1 << 20) / float(np.mean(v)), len(v)  # KiB expected per 1 GiB copy

        ff, nf = factor(args.copy_fetch_csv, "FETCH_SIZE")
        wf, nw = factor(args.copy_write_csv, "WRITE_SIZE")
        fetch = np.array(_counter_per_dispatch(args.fetch_csv, "FETCH_SIZE", kname))
        write = np.array(_counter_per_dispatch(args.write_csv, "WRITE_SIZE", kname))
        assert len(fetch) == len(write) == len(pushes), (len(fetch), len(write), len(pushes))
        fb = fetch * ff * 1024.0
        wb = write * wf * 1024.0
        alg_step = (np.array(cp["alg_bytes_per_step"], dtype=float) if "alg_bytes_per_step" in cp
                    else pushes * bpp)
        traffic = float(np.mean(fb + wb))
        prof["pmc"] = {"steps": int(len(pushes)), "fetch_factor": ff, "write_factor": wf,
                       "copy_dispatches": [nf, nw],
                       "fetch_bytes_per_launch": float(np.mean(fb)),
                       "write_bytes_per_launch": float(np.mean(wb)),
                       "traffic_bytes_per_launch": traffic,
                       "alg_bytes_per_launch": float(np.mean(alg_step)),
                       "traffic_over_alg": traffic / float(np.mean(alg_step)),
                       "per_step_ratio": [float(x) for x in (fb + wb) / alg_step]}
        lines += ["", f"## HBM traffic of {kname} (counter passes over the first {len(pushes)} steps, "
                      "one counter per run)", "",
                  f"- calibration: 1 GiB device copies read FETCH_SIZE {1024 * 1024 / ff:.0f} KiB and "
                  f"write WRITE_SIZE {1024 * 1024 / wf:.0f} KiB each (factors {ff:.3f}, {wf:.3f})",
                  f"- per launch, averaged over the {len(pushes)} steps: read {np.mean(fb) / 1e6:.2f} MB, "
                  f"written {np.mean(wb) / 1e6:.2f} MB, total {traffic / 1e6:.2f} MB against "
                  f"{np.mean(alg_step) / 1e6:.2f} MB algorithmic ({bpp} B per push, {BYTES_PER_PHOTON} B per photon emitted): ratio "
                  f"{traffic / np.mean(alg_step):.3f}", "",
                  "| step | leptons pushed | read MB | written MB | traffic / algorithmic |",
                  "|---|---|---|---|---|"]
        lines += [f"| {k + 1} | {int(pushes[k])} | {fb[k] / 1e6:.2f} | {wb[k] / 1e6:.2f} | "
                  f"{(fb[k] + wb[k]) / alg_step[k]:.3f} |" for k in range(len(pushes))]
    if args.lds_csv:
        conf = np.array(_counter_per_dispatch(args.lds_csv, "SQ_LDS_BANK_CONFLICT", kname))
        insts = np.array(_counter_per_dispatch(args.lds_csv, "SQ_INSTS_LDS", kname))
        prof["pmc"]["lds_bank_conflict_cycles_per_lds_inst"] = float(conf.sum() / max(insts.sum(), 1))
        lines += ["", "## LDS (flux tile, emitter list)", "",
                  f"- SQ_LDS_BANK_CONFLICT {conf.sum():.0f} cycles over SQ_INSTS_LDS {insts.sum():.0f} "
                  f"instructions: {conf.sum() / max(insts.sum(), 1):.3f} conflict cycles per LDS instruction"]
    base = os.path.join(PROFILE_DIR, _profile_name(workload, prec))
    os.makedirs(PROFILE_DIR, exist_ok=True)
    with open(base + ".json", "w") as f:
        json.dump(prof, f, indent=1)
    lines += [""] + [f"Note: {n}" for n in args.note] + ([""] if args.note else [])
    with open(base + ".md", "w") as f:
        f.write("\n".join(lines))
    print(base + ".md")


def host_cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), for the CPU baseline."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _leg(r, precision):
    leg = dict(value=r["pushes"] / r["seconds"], unit="pushes/s", pushes=r["pushes"],
               seconds=r["seconds"], steps=r["steps"], frozen_gaps=r["frozen"],
               run_seconds=r["run_seconds"])
    if r["push_ms"]:
        leg["push_kernel_GBs"] = r["evented_bytes"] / (r["push_ms"] * 1e-3) / 1e9
    return leg


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: whole job)")
    ap.add_argument("--warmup", type=int, default=5,
                    help="untimed steps of a throwaway batch of the same workload first")
    ap.add_argument("--reps", type=int, default=5,
                    help="timed runs on fresh batches; the median is reported")
    ap.add_argument("--workload", default="c4_batched",
                    choices=["c4_batched", "n1_corotating", "n3_uniform", "n4_spread", "n4_spline",
                             "n4_nonuniform", "ubench_lattice"]
                    + sorted(workloads.CONFIGS))
    ap.add_argument("--sort-every", type=int, default=None,
                    help="re-sort cadence for every gap (0 = tuned while running; default: the workload's)")
    ap.add_argument("--cpu-gaps", type=int, default=32)
    ap.add_argument("--cpu-steps", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the comparison legs")
    ap.add_argument("--dump-history", default=None, help="save the history rows (.npy, single gap)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy a 1 GiB device buffer 3 times (counter calibration)")
    ap.add_argument("--counter-pass", type=int, default=0, metavar="STEPS",
                    help="only run the first STEPS steps eagerly, one line per step (PMC passes)")
    ap.add_argument("--timed-only", action="store_true",
                    help="skip the evented rerun (counter passes: same push dispatches, graph-replayed)")
    ap.add_argument("--summarize", action="store_true",
                    help="write the profiles/ summary from rocprofv3 CSV output (no GPU)")
    ap.add_argument("--bench-json")
    ap.add_argument("--trace-csv")
    ap.add_argument("--pmc-json", help="output of the --counter-pass run")
    ap.add_argument("--fetch-csv")
    ap.add_argument("--write-csv")
    ap.add_argument("--lds-csv")
    ap.add_argument("--copy-fetch-csv")
    ap.add_argument("--copy-write-csv")
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--note", action="append", default=[])
    args = ap.parse_args()
    if args.summarize:
        summarize(args)
        return
    if args.gpus != 1:
        print(f"bench.py: this path runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent gaps would shard across GPUs without communication; not built here)",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        import torch
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 1 << 30, "copies": 3}))
        return

    gaps = _workload(args.workload)
    if args.sort_every is not None:
        gaps = [dict(c, sort_every=args.sort_every) for c in gaps]
    if args.counter_pass:
        run_counter_pass(gaps, args.counter_pass)
        return
    prec = gaps[0]["precision"]
    steps = args.steps if args.steps is not None else DEFAULT_STEPS.get(args.workload, gaps[0]["steps"])

    # the oracle's process pool forks before anything touches the GPU
    cpu = None
    if not args.no_cpu:
        sample = gaps[:args.cpu_gaps]
        procs = min(len(sample), os.cpu_count() or 1, 16)
        # a bounded sample of 10-30 s of oracle work, whatever the timed steps
        cb = run_cpu_baseline(sample, args.cpu_steps, procs)
        cpu = dict(value=cb["value"], unit="pushes/s", cores=procs, kind="oracle",
                   sample=f"first {args.cpu_steps} steps of {len(sample)} gap(s) of "
                          f"{args.workload}, one gap per process ({cb['pushes']} pushes, "
                          f"{cb['seconds']:.1f} s)",
                   host_nproc=os.cpu_count(), host_cpu=host_cpu_model())

    copy_gbs = None if args.timed_only else measure_copy_gbs()
    main_run = run_gpu(gaps, steps, warmup=args.warmup, reps=args.reps,
                       profile=not args.timed_only, dump=args.dump_history)
    value = main_run["pushes"] / main_run["seconds"]
    bpp = BYTES_PER_PUSH[prec]
    if args.timed_only:
        print(json.dumps({"timed_only": True, "workload": args.workload, "steps": main_run["steps"],
                          "pushes": main_run["pushes"], "value": value}), flush=True)
        return
    achieved = main_run["evented_bytes"] / (main_run["push_ms"] * 1e-3) / 1e9

    extra = {}
    if not args.no_compare:
        if args.workload == "c4_batched":
            r = run_gpu(_workload("c4_batched", workloads.FP64), steps, warmup=args.warmup,
                        reps=args.reps, profile=False)
            extra["fp64_batched_same_workload"] = _leg(r, workloads.FP64)
            c2 = _workload("c2_fp64_single_gap")
            r = run_gpu(c2, DEFAULT_STEPS["c2_fp64_single_gap"], warmup=args.warmup, reps=1,
                        profile=True)
            leg = _leg(r, workloads.FP64)
            leg["workload"] = "c2_fp64_single_gap (8192 cells, 1024 seed pairs, first 10000 steps)"
            extra["plain_fp64_single_gap"] = leg
        elif prec == workloads.FP64:
            r = run_gpu(_workload(args.workload, workloads.MIXED), steps, warmup=args.warmup,
                        reps=args.reps, profile=True)
            extra["mixed_same_workload"] = _leg(r, workloads.MIXED)

    pmc = stored_traffic(args.workload, prec, steps)
    tu = main_run["tuning"]
    cfg = {"workload": args.workload, "gaps": len(gaps), "steps": steps,
           "pushes": main_run["pushes"], "frozen_gaps": main_run["frozen"],
           "frozen": [{"gap": i, "status": st, "steps_done": n} for i, st, n in main_run["frozen_gaps"]],
           "timed_runs": {"reps": args.reps, "statistic": "median",
                          "seconds": main_run["run_seconds"],
                          "prepare_seconds": main_run["prepare_s"],
                          "warmup_steps": args.warmup},
           "sort_every": {"autotuned": tu["autotuned"], "final": tu["sort_every"],
                          "switches": tu["switches"], "timed_replays": tu["replays"]}}
    if len(gaps) == 1:
        cfg.update(n_cells=gaps[0]["n_cells"], seed_pairs=gaps[0]["n_pairs"], e0=gaps[0]["e0"],
                   gamma_thr=gaps[0]["gamma_thr"], l_gamma=gaps[0]["l_gamma"],
                   peak_leptons=main_run["peak_leptons"])
        if args.workload in ("n3_uniform", "n4_spread", "n4_spline"):
            cfg.update(f=gaps[0]["f"], dt=gaps[0]["dt"], dx=gaps[0]["dx"], boundary="periodic",
                       gamma_thr_spread=gaps[0].get("gamma_thr_spread", 0.0),
                       shape="quadratic spline" if gaps[0].get("shape") else "cloud in cell",
                       seed="one pair per cell at rest, random positions")
        if gaps[0].get("E_init") is not None:
            cfg.update(e_profile="E0 exp(-x / (L/4)) from the surface wall", dt=gaps[0]["dt"],
                       dx=gaps[0]["dx"], f=gaps[0]["f"],
                       seed="pairs at rest, density exp(-x / (L/4)), mean 1 per cell")
        if gaps[0].get("j_m"):
            cfg.update(j_m=gaps[0]["j_m"], dt=gaps[0]["dt"], dx=gaps[0]["dx"], f=gaps[0]["f"],
                       seed="cold streams: electrons at density 2, -0.5 c; positrons at 1, +0.5 c")
    else:
        cfg.update(n_cells="log-uniform 1024-16384", e0="U[50,400]", gamma_thr="U[50,400]",
                   l_gamma="U[10,100] cells", seed_pairs="log-uniform 256-4096",
                   caps="1e5-1e7 per species")
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "pushes/s",
        "n_gpus": 1,
        "steps": main_run["steps"],
        "warmup": args.warmup,
        "ms_per_step": main_run["seconds"] * 1e3 / max(main_run["steps"], 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec],
        "data": "synthetic",
        "config": cfg,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": pmc["traffic_bytes_per_launch"] if pmc else None,
                     "traffic_unit": "B/launch",
                     "alg_bytes_per_launch": main_run["evented_bytes"] / max(main_run["push_launches"], 1),
                     "evented_run": {"pushes": main_run["evented_pushes"],
                                     "push_emissions": main_run["evented_photons"],
                                     "sort_every": main_run["evented_tuning"]["sort_every"],
                                     "switches": main_run["evented_tuning"]["switches"]},
                     "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                     "kernel": "k_push", "bytes_per_push": bpp, "bytes_per_photon": BYTES_PER_PHOTON,
                     "kernel_ms": main_run["push_ms"], "launches": main_run["push_launches"]},
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
