"""Oracle for the 1D pair-cascade PIC step -- TEST INFRASTRUCTURE ONLY.

A ctypes wrapper around ``libpic_oracle.so`` (plain scalar C, see
``pic_oracle.c``).  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product path never does.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

FP64, MIXED = 0, 1
PERIODIC, ABSORBING = 0, 1
SEED_RANDOM, SEED_LATTICE = 0, 1
SHAPE_LINEAR, SHAPE_QUADRATIC = 0, 1
OK, ERR_ARG, ERR_CAPACITY, ERR_STATE, ERR_NONFINITE, ERR_EMISSION = 0, -1, -3, -5, -6, -7


class Params(C.Structure):
    _fields_ = [
        ("n_cells", C.c_int32), ("dx", C.c_double), ("dt", C.c_double),
        ("boundary", C.c_int32), ("e0", C.c_double), ("gamma_thr", C.c_double),
        ("f", C.c_double), ("l_gamma", C.c_double), ("weight", C.c_double),
        ("seed", C.c_uint64), ("precision", C.c_int32), ("capacity", C.c_int64),
        ("j_m", C.c_double), ("gamma_thr_spread", C.c_double), ("shape", C.c_int32),
    ]


class HistoryRow(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("n_minus", C.c_int64), ("n_plus", C.c_int64),
        ("n_photons", C.c_int64), ("pairs_created", C.c_int64),
        ("photons_emitted", C.c_int64), ("photons_escaped", C.c_int64),
        ("absorbed_minus", C.c_int64), ("absorbed_plus", C.c_int64),
        ("kinetic", C.c_double), ("field", C.c_double), ("photon_energy", C.c_double),
        ("lost_energy", C.c_double), ("e_mean", C.c_double),
    ]


HISTORY_DTYPE = np.dtype([(n, np.int64 if t is C.c_int64 else np.float64)
                          for n, t in HistoryRow._fields_])


def lib():
    """Loads the oracle library, building it first if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(_HERE, "libpic_oracle.so")
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
        _build.build()
    L = C.CDLL(path)
    vp, i32, i64, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    P = C.POINTER
    L.orc_validate.argtypes = [P(Params)]; L.orc_validate.restype = C.c_int
    L.orc_create.argtypes = [P(Params)]; L.orc_create.restype = vp
    L.orc_destroy.argtypes = [vp]; L.orc_destroy.restype = None
    L.orc_seed.argtypes = [vp, i32, i64, i32, dbl, dbl]; L.orc_seed.restype = C.c_int
    L.orc_seed_explicit.argtypes = [vp, i32, i64, vp, vp, vp, vp]
    L.orc_seed_explicit.restype = C.c_int
    L.orc_step.argtypes = [vp, i64]; L.orc_step.restype = C.c_int
    L.orc_status.argtypes = [vp]; L.orc_status.restype = C.c_int
    L.orc_steps_done.argtypes = [vp]; L.orc_steps_done.restype = i64
    L.orc_count.argtypes = [vp, i32]; L.orc_count.restype = i64
    L.orc_photon_count.argtypes = [vp]; L.orc_photon_count.restype = i64
    L.orc_read_particles.argtypes = [vp, i32, i64, vp, vp, vp, vp, P(i64)]
    L.orc_read_particles.restype = C.c_int
    L.orc_read_photons.argtypes = [vp, i64, vp, vp, vp, vp, P(i64)]
    L.orc_read_photons.restype = C.c_int
    L.orc_read_fields.argtypes = [vp, vp, vp, vp]; L.orc_read_fields.restype = C.c_int
    L.orc_set_fields.argtypes = [vp, vp]; L.orc_set_fields.restype = C.c_int
    L.orc_history.argtypes = [vp, vp, i64, P(i64)]; L.orc_history.restype = C.c_int
    L.orc_offset_bits.argtypes = [vp]; L.orc_offset_bits.restype = C.c_int
    L.orc_event_map.argtypes = [vp, i32, i32, i32]; L.orc_event_map.restype = C.c_int
    L.orc_read_event_map.argtypes = [vp, vp]; L.orc_read_event_map.restype = C.c_int
    L.orc_philox4x64_10.argtypes = [vp, vp, vp]; L.orc_philox4x64_10.restype = None
    L.orc_philox4x32_10.argtypes = [vp, vp, vp]; L.orc_philox4x32_10.restype = None
    L.orc_conv_table.argtypes = [dbl, dbl, dbl, vp, i64]; L.orc_conv_table.restype = i64
    _LIB = L
    return L


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def make_params(n_cells, dx, dt, boundary, e0, gamma_thr, f, l_gamma, weight, seed,
                precision=FP64, capacity=0, j_m=0.0, gamma_thr_spread=0.0, shape=0):
    return Params(n_cells, dx, dt, boundary, e0, gamma_thr, f, l_gamma, weight, seed,
                  precision, capacity, j_m, gamma_thr_spread, shape)


def validate(**kw):
    return lib().orc_validate(C.byref(make_params(**kw)))


def philox4x64_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint64).copy()
    k = np.asarray(key, dtype=np.uint64).copy()
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def conv_table(dt, dx, l_gamma):
    L = lib()
    n = L.orc_conv_table(dt, dx, l_gamma, None, 0)
    t = np.zeros(max(n, 0), dtype=np.uint32)
    if n > 0:
        L.orc_conv_table(dt, dx, l_gamma, _ptr(t), n)
    return t


class OracleGap:
    """One gap advanced by the oracle; mirrors the library's call sequence."""

    def __init__(self, **kw):
        self.params = make_params(**kw)
        self._L = lib()
        h = self._L.orc_create(C.byref(self.params))
        if not h:
            raise ValueError("oracle rejected the parameters")
        self._h = h
        self.n_cells = self.params.n_cells

    def close(self):
        if self._h:
            self._L.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def offset_bits(self):
        return self._L.orc_offset_bits(self._h)

    def seed(self, mode, n_pairs, macro_per_pair=1, p0_minus=0.0, p0_plus=0.0):
        st = self._L.orc_seed(self._h, mode, n_pairs, macro_per_pair, p0_minus, p0_plus)
        if st != OK:
            raise RuntimeError(f"orc_seed failed: {st}")

    def seed_explicit(self, species, cell, off, p, ids):
        cell = np.ascontiguousarray(cell, dtype=np.int32)
        off = np.ascontiguousarray(off, dtype=np.float64)
        p = np.ascontiguousarray(p, dtype=np.float64)
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        st = self._L.orc_seed_explicit(self._h, species, len(cell), _ptr(cell), _ptr(off),
                                       _ptr(p), _ptr(ids))
        if st != OK:
            raise RuntimeError(f"orc_seed_explicit failed: {st}")

    def step(self, n):
        return self._L.orc_step(self._h, n)

    @property
    def status(self):
        return self._L.orc_status(self._h)

    @property
    def steps_done(self):
        return self._L.orc_steps_done(self._h)

    def count(self, species):
        return self._L.orc_count(self._h, species)

    def photon_count(self):
        return self._L.orc_photon_count(self._h)

    def particles(self, species):
        n = self.count(species)
        cell = np.zeros(n, np.int32); off = np.zeros(n); p = np.zeros(n)
        ids = np.zeros(n, np.uint64); n_out = C.c_int64()
        self._L.orc_read_particles(self._h, species, n, _ptr(cell), _ptr(off), _ptr(p),
                                   _ptr(ids), C.byref(n_out))
        return {"cell": cell, "off": off, "p": p, "id": ids}

    def photons(self):
        n = self.photon_count()
        xq = np.zeros(n, np.int64); cs = np.zeros(n, np.int64)
        d = np.zeros(n, np.int32); ch = np.zeros(n, np.uint64); n_out = C.c_int64()
        self._L.orc_read_photons(self._h, n, _ptr(xq), _ptr(cs), _ptr(d), _ptr(ch),
                                 C.byref(n_out))
        return {"xq": xq, "conv_step": cs, "dir": d, "child": ch}

    def fields(self):
        E = np.zeros(self.n_cells); rho = np.zeros(self.n_cells + 1)
        F = np.zeros(self.n_cells, np.int64)
        self._L.orc_read_fields(self._h, _ptr(E), _ptr(rho), _ptr(F))
        return {"E": E, "rho": rho, "flux": F}

    def event_map(self, x_bins, steps_per_row, rows):
        """Starts counting pair events by (step row, cell bin)."""
        st = self._L.orc_event_map(self._h, x_bins, steps_per_row, rows)
        if st != OK:
            raise RuntimeError(f"orc_event_map failed: {st}")
        self._ev = (x_bins, rows)

    def read_event_map(self):
        x_bins, rows = self._ev
        out = np.zeros((rows, x_bins), np.int64)
        st = self._L.orc_read_event_map(self._h, _ptr(out))
        if st != OK:
            raise RuntimeError(f"orc_read_event_map failed: {st}")
        return out

    def set_fields(self, E):
        E = np.ascontiguousarray(E, dtype=np.float64)
        st = self._L.orc_set_fields(self._h, _ptr(E))
        if st != OK:
            raise RuntimeError(f"orc_set_fields failed: {st}")

    def history(self):
        n_out = C.c_int64()
        self._L.orc_history(self._h, None, 0, C.byref(n_out))
        rows = (HistoryRow * max(n_out.value, 1))()
        self._L.orc_history(self._h, C.cast(rows, C.c_void_p), n_out.value, C.byref(n_out))
        buf = np.frombuffer(bytes(rows), dtype=HISTORY_DTYPE, count=n_out.value)
        return buf.copy()
