"""The C-ABI library on the host: it loads, exports every function that
include/pic.h declares, and validates parameters and workspaces without
touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads
from tests import pic_cases as pc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pic.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pic_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    import paper_2012_05587_amd as P
    L = P.lib()
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(P.EXPORTS)


def test_binding_fails_loudly_without_library(monkeypatch):
    import paper_2012_05587_amd as P
    monkeypatch.setattr(P, "_lib", None)
    monkeypatch.setattr(P, "LIB_PATH", os.path.join(ROOT, "no_such_lib.so"))
    with pytest.raises(RuntimeError):
        P.lib()


def _valid():
    return dict(workloads.config("c1_fp64_reference_gap"))


def test_validate_accepts_configs():
    import paper_2012_05587_amd as P
    for name in workloads.CONFIGS:
        assert P.pic_validate_params(pc.gpu_params(workloads.config(name))) == P.OK, name
    for c in workloads.batched_scan(n_gaps=16):
        assert P.pic_validate_params(pc.gpu_params(c)) == P.OK


@pytest.mark.parametrize("field,value", [
    ("dt", 1.0), ("dt", -0.1), ("n_cells", 1), ("boundary", 5), ("f", 0.0), ("f", 1.0),
    ("f", 0.01), ("gamma_thr", 1.0), ("l_gamma", -2.0), ("weight", -1.0), ("capacity", 0),
    ("capacity", 2**31), ("precision", 3), ("e0", float("inf")), ("sort_every", -1),
    ("j_m", float("nan")), ("gamma_thr_spread", -0.1), ("gamma_thr_spread", 1.0),
    ("gamma_thr_spread", 0.5), ("shape", 2), ("shape", -1), ("l_gamma", 1e30),
    ("n_cells", 2**22 + 1),
])
def test_validate_rejects(field, value):
    import paper_2012_05587_amd as P
    c = _valid()
    c[field] = value
    assert P.pic_validate_params(pc.gpu_params(c)) == P.ERR_ARG
    assert P.pic_workspace_bytes(pc.gpu_params(c)) == 0


def test_variants_validate_alike_in_library_and_oracle():
    """The library and the oracle accept and reject the same variant
    parameters: a spread of gamma_thr needs (1 - f - sigma) gamma_thr >= 1,
    the quadratic shape at least 4 cells."""
    import oracle

    import paper_2012_05587_amd as P
    cases = []
    for spread in (0.0, 0.2, 0.49, 0.5, 0.99):
        for shape in (0, 1):
            for bc in (workloads.PERIODIC, workloads.ABSORBING):
                for nc in (3, 4, 512):
                    cases.append(dict(_valid(), gamma_thr_spread=spread, shape=shape,
                                      boundary=bc, n_cells=nc))
    accepted = 0
    for c in cases:
        lib_ok = P.pic_validate_params(pc.gpu_params(c)) == P.OK
        orc_ok = oracle.validate(**pc.gap_kwargs(c)) == oracle.OK
        assert lib_ok == orc_ok, c
        accepted += lib_ok
    assert 0 < accepted < len(cases)


def test_position_range_validates_alike_in_library_and_oracle():
    """Positions are int64 multiples of 2^-K cells: the domain and a
    photon's longest path (where its conversion table ends, about 22.2
    l_gamma cells) must each stay below 2^62 of them.  In binary64 (K = 40)
    that caps n_cells at 2^22 and l_gamma near 1.9e5 cells; the 2^-24 grid of
    the mixed path leaves room for far longer paths."""
    import oracle

    import paper_2012_05587_amd as P
    verdicts = {}
    for prec in (workloads.FP64, workloads.MIXED):
        for l_gamma in (20.0, 1.8e5, 2.0e5, 1e6):
            for nc in (512, 2**22):
                c = dict(_valid(), precision=prec, l_gamma=l_gamma, n_cells=nc,
                         photon_capacity=1000)
                lib_ok = P.pic_validate_params(pc.gpu_params(c)) == P.OK
                orc_ok = oracle.validate(**pc.gap_kwargs(c)) == oracle.OK
                assert lib_ok == orc_ok, c
                verdicts[(prec, l_gamma, nc)] = lib_ok
    assert verdicts[(workloads.FP64, 1.8e5, 512)]
    assert not verdicts[(workloads.FP64, 2.0e5, 512)]
    assert not verdicts[(workloads.FP64, 1e6, 512)]
    assert verdicts[(workloads.MIXED, 1e6, 512)]
    assert verdicts[(workloads.FP64, 20.0, 2**22)]
    # the longest path and the domain are bounded separately
    assert verdicts[(workloads.FP64, 1.8e5, 2**22)]


def test_photon_store_required_for_finite_path():
    import paper_2012_05587_amd as P
    c = _valid()
    c["photon_capacity"] = 0
    assert P.pic_validate_params(pc.gpu_params(c)) == P.ERR_ARG
    c["l_gamma"] = 0.0
    assert P.pic_validate_params(pc.gpu_params(c)) == P.OK


def test_workspace_grows_with_capacity_and_precision():
    import paper_2012_05587_amd as P
    c = _valid()
    a = P.pic_workspace_bytes(pc.gpu_params(c))
    b = P.pic_workspace_bytes(pc.gpu_params(c, capacity=2 * c["capacity"]))
    m = P.pic_workspace_bytes(pc.gpu_params(c, precision=workloads.MIXED))
    assert 0 < a < b and m < a
    # per-slot bytes: 2 buffers x 2 species x (4 + 8 + 8 + 8) in binary64, plus a
    # 4-byte emission-list entry per species; capacity + capacity/8 + 2048 slots
    slots = lambda cap: cap + cap // 8 + 2048  # noqa: E731
    extra = slots(2 * c["capacity"]) - slots(c["capacity"])
    assert abs((b - a) - (2 * 2 * 28 + 8) * extra) <= 16 * 1024


def test_batch_plan_admits_under_budget():
    import paper_2012_05587_amd as P
    gaps = [pc.gpu_params(c) for c in workloads.batched_scan(n_gaps=32)]
    full = P.lib().pic_batch_workspace_bytes((P.GapParams * 32)(*gaps), 32)
    adm, ws = P.batch_plan(gaps, full)
    assert adm.all() and ws == full
    adm, ws = P.batch_plan(gaps, full // 3)
    assert 0 < adm.sum() < 32 and ws <= full // 3


def test_batch_slot_limit():
    """A batch holds fewer than 2^32 lepton slots (both species); a species
    fewer than 2^31 (capacity + capacity/8 + 2048)."""
    import paper_2012_05587_amd as P
    cmax = ((1 << 31) - 1 - 2048) * 8 // 9
    assert P.pic_validate_params(pc.gpu_params(_valid(), capacity=cmax, photon_capacity=1)) == P.OK
    assert P.pic_validate_params(pc.gpu_params(_valid(), capacity=cmax + 8, photon_capacity=1)) == P.ERR_ARG
    big = pc.gpu_params(_valid(), capacity=cmax, photon_capacity=1)
    two = (P.GapParams * 2)(big, big)
    assert P.lib().pic_batch_workspace_bytes(two, 2) == 0
    assert P.lib().pic_batch_workspace_bytes((P.GapParams * 1)(big), 1) > 0
    adm, _ = P.batch_plan([big, big], 1 << 62)
    assert list(adm) == [1, 0]


def test_create_rejects_bad_workspace_without_device():
    import paper_2012_05587_amd as P
    prm = pc.gpu_params(_valid())
    h = C.c_void_p()
    assert P.lib().pic_create_gap(C.byref(prm), None, 1 << 30, None, C.byref(h)) == P.ERR_WORKSPACE
    assert P.lib().pic_create_gap(C.byref(prm), C.c_void_p(256), 16, None, C.byref(h)) == P.ERR_WORKSPACE
    assert P.lib().pic_create_gap(C.byref(prm), C.c_void_p(4096 + 8), 1 << 40, None,
                                  C.byref(h)) == P.ERR_WORKSPACE


def test_emission_split_rejects_null_handles():
    import paper_2012_05587_amd as P
    assert P.lib().pic_emission_split(None, 0) == P.ERR_ARG
    assert P.lib().pic_batch_emission_split(None, 32768) == P.ERR_ARG


def test_status_strings():
    import paper_2012_05587_amd as P
    for st in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert P.status_string(st)
    assert "unknown" in P.status_string(-99)


def test_oracle_and_library_share_no_code():
    """The oracle sources name nothing from the HIP library and vice versa."""
    orc = open(os.path.join(ROOT, "oracle", "pic_oracle.c")).read()
    assert "pic.h" not in orc and "pic_device" not in orc
    for f in os.listdir(os.path.join(ROOT, "paper_2012_05587_amd", "csrc")):
        if f.endswith((".hip", ".cpp", ".hpp")):
            txt = open(os.path.join(ROOT, "paper_2012_05587_amd", "csrc", f)).read()
            assert "pic_oracle" not in txt and "orc_" not in txt, f
    for f in ("__init__.py", "build.py"):
        txt = open(os.path.join(ROOT, "paper_2012_05587_amd", f)).read()
        assert "import oracle" not in txt and "from oracle" not in txt
