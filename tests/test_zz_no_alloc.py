"""The allocation-free read of the fields (pic_read_fields_noalloc) against
pic_read_fields, through the C-ABI (needs a GPU).

Two calls in a row on the static node scratch, the second on a smaller gap,
must give E and rho bit for bit as the workspace path does (the charge is an
exact integer sum on both); a gap beyond the static array's 2^20 + 1 nodes
is refused when rho is asked for, and still reads E.
"""
import ctypes as C

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


def _read(P, gg, fn):
    n = gg.n_cells
    E = np.full(n, np.nan)
    rho = np.full(n + 1, np.nan)
    st = getattr(P.lib(), fn)(gg._h, E.ctypes.data_as(C.c_void_p), rho.ctypes.data_as(C.c_void_p), n)
    return st, E, rho


def test_noalloc_read_matches_workspace_read():
    import paper_2012_05587_amd as P
    big = workloads.config("c1_fp64_reference_gap")
    small = dict(big, n_cells=96, n_pairs=40, macro_per_pair=2, seed=big["seed"] + 1,
                 boundary=workloads.PERIODIC, precision=workloads.MIXED)
    for cfg, steps in ((big, 300), (small, 80)):
        print(f"[case] noalloc read {cfg['n_cells']} cells, {steps} steps", flush=True)
        gg = pc.make_gpu(cfg)
        gg.step_n(steps)
        st0, E0, r0 = _read(P, gg, "pic_read_fields")
        st1, E1, r1 = _read(P, gg, "pic_read_fields_noalloc")
        assert st0 == P.OK and st1 == P.OK
        assert np.array_equal(E0, E1)
        assert np.array_equal(r0, r1)
        assert np.abs(r1).max() > 0
        # E alone, rho not requested
        E2 = np.zeros(gg.n_cells)
        assert P.lib().pic_read_fields_noalloc(gg._h, E2.ctypes.data_as(C.c_void_p), None,
                                               gg.n_cells) == P.OK
        assert np.array_equal(E2, E0)
        # and Gauss's law on the charge it returns
        r = pc.gauss_residual(E1, r1, periodic=cfg["boundary"] == workloads.PERIODIC)
        assert np.abs(r).max() <= 10 * np.finfo(float).eps * steps * np.abs(E1).max()
        gg.close()


def test_noalloc_read_refuses_more_nodes_than_its_scratch():
    import paper_2012_05587_amd as P
    cfg = dict(n_cells=(1 << 20) + 1, dx=1.0, dt=0.45, boundary=workloads.ABSORBING, e0=5.0,
               gamma_thr=100.0, f=0.5, l_gamma=0.0, weight=1.0, seed=3, precision=workloads.FP64,
               n_pairs=16, macro_per_pair=1, capacity=4096, photon_capacity=0)
    gg = pc.make_gpu(cfg)
    gg.step_n(2)
    st, E, rho = _read(P, gg, "pic_read_fields_noalloc")
    assert st == P.ERR_ARG
    E2 = np.zeros(gg.n_cells)
    assert P.lib().pic_read_fields_noalloc(gg._h, E2.ctypes.data_as(C.c_void_p), None,
                                           gg.n_cells) == P.OK
    assert np.array_equal(E2, gg.read_fields(rho=False)["E"])
    gg.close()
