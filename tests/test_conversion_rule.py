"""The HIP path decides a photon's conversion step without its table where a
binary32 evaluation provably gives the table's answer (CPU test of that rule).

n_conv = min{k >= 1 : u >= T_k} with T_k = floor(2^32 q^k), q = exp(-r),
r = dt / (l_gamma dx) (the finite photon path; each step the photon survives
with probability q).  For an integer u, u >= floor(V) exactly when u + 1 > V,
so n_conv = floor(x) + 1 with x = (32 - log2(u + 1)) ln 2 / r.  The kernel
evaluates x in binary32 and accepts floor(x) + 1 only when x lies farther than
tol = 2e-5 c + 5e-7 x + 1e-6 (c = ln 2 / r) from an integer; otherwise it
reads the table.  This test restates that rule in numpy binary32, with the
logarithm moved by one ulp either way (the device's log2f is within one ulp),
and checks every accepted answer against the oracle's table, on random draws
and on draws next to every table entry."""
import math

import numpy as np
import pytest

import oracle


def _rule(u, c, nt, ulp):
    y = (u.astype(np.uint64) + np.uint64(1)).astype(np.float32)
    lg = np.log2(y).astype(np.float32)
    if ulp:
        lg = np.nextafter(lg, np.float32(np.inf if ulp > 0 else -np.inf))
    x = ((np.float32(32.0) - lg).astype(np.float32) * c).astype(np.float32)
    fl = np.floor(x)
    fr = (x - fl).astype(np.float32)
    tol = (np.float32(2e-5) * c + np.float32(5e-7) * x + np.float32(1e-6)).astype(np.float32)
    ok = (fr > tol) & (fr < np.float32(1.0) - tol) & (fl + np.float32(1.0) < np.float32(nt))
    return ok, fl.astype(np.int64) + 1


def _exact(table, u):
    # first k >= 1 with T_k <= u (T decreasing to 0)
    neg = -table[1:].astype(np.float64)
    return np.searchsorted(neg, -u.astype(np.float64), side="left") + 1


@pytest.mark.parametrize("dt,dx,l_gamma", [(0.45, 1.0, 10.0), (0.45, 1.0, 20.0), (0.45, 1.0, 100.0),
                                           (0.99, 1.0, 10.0), (1e-3, 0.1, 5.0),
                                           (3.16e-4, 0.0158, 0.5), (0.45, 1.0, 1e4)])
def test_direct_conversion_rule_matches_table(dt, dx, l_gamma):
    table = np.array(oracle.conv_table(dt, dx, l_gamma), dtype=np.uint64)
    nt = len(table)
    c = np.float32(math.log(2.0) * l_gamma * dx / dt)
    rng = np.random.default_rng(int(l_gamma * 1000 + dt * 1e4))
    u = [rng.integers(0, 2**32, 100000, dtype=np.uint64)]
    ks = rng.integers(1, nt, 3000)
    near = (table[ks][:, None].astype(np.int64) + np.arange(-2, 3)[None, :]).ravel()
    u.append(near[(near >= 0) & (near < 2**32)].astype(np.uint64))
    u.append(np.array([0, 1, 2**32 - 2, 2**32 - 1], dtype=np.uint64))
    u = np.concatenate(u)
    exact = _exact(table, u)
    accepted = 0
    for ulp in (-1, 0, 1):
        ok, n = _rule(u, c, nt, ulp)
        bad = ok & (n != exact)
        assert not bad.any(), (u[bad][:5], n[bad][:5], exact[bad][:5])
        accepted += int(ok.sum())
    # the rule answers most draws (the table is read only near integers)
    if l_gamma * dx / dt < 1e3:
        assert accepted > 0.9 * 3 * len(u)
