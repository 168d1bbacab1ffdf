"""Python binding of libpic_cascade.so: the MI355X pair-cascade PIC step.

Argument marshalling only.  Every step of the path runs in the library's HIP
kernels; PyTorch supplies the device workspace and the stream.  The names
follow the C-ABI in include/pic.h (``pic_create_gap``, ``pic_seed_particles``,
``pic_step_n``, ``pic_read_fields``, ``pic_read_moments``, ``pic_destroy``, ...),
and ``Gap`` / ``Batch`` wrap them for convenience.

The library is loaded from this directory; if it is missing, importing the
path raises: there is no fallback.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic_cascade.so")

OK, ERR_ARG, ERR_WORKSPACE, ERR_CAPACITY, ERR_DEVICE, ERR_STATE, ERR_NONFINITE, ERR_EMISSION = \
    0, -1, -2, -3, -4, -5, -6, -7
ERR_SLOTS = -8
BC_PERIODIC, BC_ABSORBING = 0, 1
FP64, MIXED = 0, 1
SEED_RANDOM, SEED_LATTICE = 0, 1
ELECTRON, POSITRON = 0, 1

EXPORTS = [
    "pic_validate_params", "pic_workspace_bytes", "pic_create_gap", "pic_seed_particles",
    "pic_seed_explicit", "pic_step_n", "pic_read_fields", "pic_read_flux", "pic_read_moments",
    "pic_read_history", "pic_read_particles", "pic_read_photons", "pic_set_fields",
    "pic_offset_bits", "pic_destroy", "pic_status_string", "pic_batch_plan",
    "pic_batch_workspace_bytes", "pic_create_batch", "pic_batch_step_n", "pic_batch_gap",
    "pic_batch_size", "pic_destroy_batch", "pic_profile_push", "pic_read_push_time",
    "pic_batch_profile_push", "pic_batch_read_push_time", "pic_batch_tuning", "pic_tuning",
    "pic_phase_space", "pic_event_map", "pic_prepare", "pic_batch_prepare",
    "pic_read_fields_noalloc", "pic_emission_split", "pic_batch_emission_split",
]


def _tuning(name, h):
    """Re-sort cadence in use: dict(sort_every, autotuned, replays, switches)."""
    se, au, rp, sw = C.c_int32(), C.c_int32(), C.c_int64(), C.c_int32()
    _check(name, getattr(lib(), name)(h, C.byref(se), C.byref(au), C.byref(rp), C.byref(sw)))
    return dict(sort_every=se.value, autotuned=bool(au.value), replays=rp.value, switches=sw.value)


class GapParams(C.Structure):
    _fields_ = [
        ("n_cells", C.c_int32), ("dx", C.c_double), ("dt", C.c_double),
        ("boundary", C.c_int32), ("e0", C.c_double), ("gamma_thr", C.c_double),
        ("f", C.c_double), ("l_gamma", C.c_double), ("weight", C.c_double),
        ("capacity", C.c_int64), ("photon_capacity", C.c_int64), ("seed", C.c_uint64),
        ("precision", C.c_int32), ("sort_every", C.c_int32), ("diag_every", C.c_int32),
        ("history_rows", C.c_int32), ("j_m", C.c_double), ("gamma_thr_spread", C.c_double),
        ("shape", C.c_int32),
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


class StepReport(C.Structure):
    _fields_ = [("steps_done", C.c_int64), ("status", C.c_int32), ("pushes", C.c_int64)]


class Moments(C.Structure):
    _fields_ = [
        ("steps_done", C.c_int64), ("status", C.c_int32), ("n_minus", C.c_int64),
        ("n_plus", C.c_int64), ("n_photons", C.c_int64), ("slots_minus", C.c_int64),
        ("slots_plus", C.c_int64), ("photon_slots", C.c_int64), ("pushes", C.c_int64),
        ("last", HistoryRow), ("push_emissions", C.c_int64),
    ]


HISTORY_DTYPE = np.dtype([(n, np.int64 if t is C.c_int64 else np.float64)
                          for n, t in HistoryRow._fields_])

_lib = None


def lib():
    """The loaded library.  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2012_05587_amd/build.py")
    # torch first: its HIP runtime is then the one the library binds to, so
    # the device memory and streams torch hands over are valid in the library
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u64, dbl, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double, C.c_size_t
    P = C.POINTER
    L.pic_validate_params.argtypes = [P(GapParams)]; L.pic_validate_params.restype = i32
    L.pic_workspace_bytes.argtypes = [P(GapParams)]; L.pic_workspace_bytes.restype = sz
    L.pic_create_gap.argtypes = [P(GapParams), vp, sz, vp, P(vp)]; L.pic_create_gap.restype = i32
    L.pic_seed_particles.argtypes = [vp, i32, i64, i32, dbl, dbl]; L.pic_seed_particles.restype = i32
    L.pic_seed_explicit.argtypes = [vp, i32, i64, vp, vp, vp, vp]; L.pic_seed_explicit.restype = i32
    L.pic_step_n.argtypes = [vp, i64, P(StepReport)]; L.pic_step_n.restype = i32
    L.pic_prepare.argtypes = [vp]; L.pic_prepare.restype = i32
    L.pic_batch_prepare.argtypes = [vp]; L.pic_batch_prepare.restype = i32
    L.pic_read_fields.argtypes = [vp, vp, vp, i32]; L.pic_read_fields.restype = i32
    L.pic_read_fields_noalloc.argtypes = [vp, vp, vp, i32]; L.pic_read_fields_noalloc.restype = i32
    L.pic_read_flux.argtypes = [vp, vp, i32]; L.pic_read_flux.restype = i32
    L.pic_read_moments.argtypes = [vp, P(Moments)]; L.pic_read_moments.restype = i32
    L.pic_read_history.argtypes = [vp, vp, i64, P(i64)]; L.pic_read_history.restype = i32
    L.pic_read_particles.argtypes = [vp, i32, i64, vp, vp, vp, vp, P(i64)]
    L.pic_read_particles.restype = i32
    L.pic_read_photons.argtypes = [vp, i64, vp, vp, vp, vp, P(i64)]; L.pic_read_photons.restype = i32
    L.pic_set_fields.argtypes = [vp, vp, i32]; L.pic_set_fields.restype = i32
    L.pic_offset_bits.argtypes = [vp]; L.pic_offset_bits.restype = i32
    L.pic_destroy.argtypes = [vp]; L.pic_destroy.restype = i32
    L.pic_status_string.argtypes = [i32]; L.pic_status_string.restype = C.c_char_p
    L.pic_batch_plan.argtypes = [P(GapParams), i32, sz, vp, P(sz)]; L.pic_batch_plan.restype = i32
    L.pic_batch_workspace_bytes.argtypes = [P(GapParams), i32]
    L.pic_batch_workspace_bytes.restype = sz
    L.pic_create_batch.argtypes = [P(GapParams), i32, vp, sz, vp, P(vp)]
    L.pic_create_batch.restype = i32
    L.pic_batch_step_n.argtypes = [vp, i64, vp]; L.pic_batch_step_n.restype = i32
    L.pic_batch_gap.argtypes = [vp, i32]; L.pic_batch_gap.restype = vp
    L.pic_batch_size.argtypes = [vp]; L.pic_batch_size.restype = i32
    L.pic_destroy_batch.argtypes = [vp]; L.pic_destroy_batch.restype = i32
    for name in ("pic_profile_push", "pic_batch_profile_push"):
        getattr(L, name).argtypes = [vp, i32]; getattr(L, name).restype = i32
    for name in ("pic_read_push_time", "pic_batch_read_push_time"):
        getattr(L, name).argtypes = [vp, P(dbl), P(i64)]; getattr(L, name).restype = i32
    L.pic_phase_space.argtypes = [vp, i32, i32, i32, dbl, dbl, vp]; L.pic_phase_space.restype = i32
    L.pic_event_map.argtypes = [vp, vp, i32, i32, i32]; L.pic_event_map.restype = i32
    for name in ("pic_tuning", "pic_batch_tuning"):
        getattr(L, name).argtypes = [vp, P(i32), P(i32), P(i64), P(i32)]; getattr(L, name).restype = i32
    for name in ("pic_emission_split", "pic_batch_emission_split"):
        getattr(L, name).argtypes = [vp, i64]; getattr(L, name).restype = i32
    _lib = L
    return L


class PicError(RuntimeError):
    def __init__(self, where, status):
        super().__init__(f"{where}: {status_string(status)} ({status})")
        self.status = status


def status_string(st):
    return lib().pic_status_string(st).decode()


def _check(where, st):
    if st != OK:
        raise PicError(where, st)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def make_params(n_cells, dx, dt, boundary, e0, gamma_thr, f, l_gamma, weight, capacity,
                photon_capacity=0, seed=0, precision=FP64, sort_every=0, diag_every=0,
                history_rows=0, j_m=0.0, gamma_thr_spread=0.0, shape=0):
    return GapParams(n_cells, dx, dt, boundary, e0, gamma_thr, f, l_gamma, weight, capacity,
                     photon_capacity, seed, precision, sort_every, diag_every, history_rows, j_m,
                     gamma_thr_spread, shape)


def pic_validate_params(params):
    return lib().pic_validate_params(C.byref(params))


def pic_workspace_bytes(params):
    return lib().pic_workspace_bytes(C.byref(params))


def _device_workspace(nbytes, device, reuse=None):
    """A uint8 device tensor of at least nbytes: `reuse` if it is large enough
    (a caller recreating gaps on the same memory), else a new one."""
    import torch
    if reuse is not None:
        if reuse.numel() < nbytes:
            raise ValueError(f"workspace of {reuse.numel()} bytes is smaller than {nbytes}")
        ws = reuse
    else:
        # 256-byte alignment is guaranteed by the caching allocator for fresh blocks
        ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace is not 256-byte aligned")
    return ws


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream), s


class _GapView:
    """Reads and seeding on one gap handle (owned or borrowed)."""

    def __init__(self, handle, params, keepalive):
        self._h = handle
        self.params = params
        self.n_cells = params.n_cells
        self._keep = keepalive

    @property
    def offset_bits(self):
        return lib().pic_offset_bits(self._h)

    def seed_particles(self, mode, n_pairs, macro_per_pair=1, p0_minus=0.0, p0_plus=0.0):
        _check("pic_seed_particles",
               lib().pic_seed_particles(self._h, mode, n_pairs, macro_per_pair, p0_minus, p0_plus))

    def seed_explicit(self, species, cell, off, p, ids):
        cell = np.ascontiguousarray(cell, np.int32); off = np.ascontiguousarray(off, np.float64)
        p = np.ascontiguousarray(p, np.float64); ids = np.ascontiguousarray(ids, np.uint64)
        _check("pic_seed_explicit", lib().pic_seed_explicit(
            self._h, species, len(cell), _ptr(cell), _ptr(off), _ptr(p), _ptr(ids)))

    def _owner(self):
        return self if self._keep is None else self._keep

    def _dev(self):
        return self._owner().workspace.device

    def _sync(self):
        """Waits for the library's stream of this gap."""
        import torch
        st = self._owner().stream
        if st is not None:
            st.synchronize()
        else:
            torch.cuda.synchronize(self._dev())

    def phase_space(self, species, x_bins, p_bins, p_min, p_max):
        """Counts of live leptons of a species by (cell bin, momentum bin), as
        an int64 array of shape (x_bins, p_bins) computed on the device."""
        import torch
        dev = self._dev()
        out = torch.zeros(x_bins * p_bins, dtype=torch.int64, device=dev)
        torch.cuda.current_stream(dev).synchronize()  # the zeros, before the library's stream
        _check("pic_phase_space", lib().pic_phase_space(
            self._h, species, x_bins, p_bins, float(p_min), float(p_max), C.c_void_p(out.data_ptr())))
        self._sync()
        return out.cpu().numpy().reshape(x_bins, p_bins)

    def set_event_map(self, x_bins, steps_per_row, rows):
        """Starts counting pair events by (step row, cell bin) on the device."""
        import torch
        m = torch.empty(rows * x_bins, dtype=torch.int64, device=self._dev())
        _check("pic_event_map", lib().pic_event_map(self._h, C.c_void_p(m.data_ptr()), x_bins,
                                                    steps_per_row, rows))
        self._evmap = (m, rows, x_bins)

    def read_event_map(self):
        m, rows, x_bins = self._evmap
        self._sync()
        return m.cpu().numpy().reshape(rows, x_bins)

    def read_fields(self, rho=True):
        E = np.zeros(self.n_cells)
        R = np.zeros(self.n_cells + 1) if rho else None
        _check("pic_read_fields", lib().pic_read_fields(self._h, _ptr(E), _ptr(R), self.n_cells))
        return {"E": E, "rho": R}

    def read_flux(self):
        F = np.zeros(self.n_cells, np.int64)
        _check("pic_read_flux", lib().pic_read_flux(self._h, _ptr(F), self.n_cells))
        return F

    def read_moments(self):
        m = Moments()
        _check("pic_read_moments", lib().pic_read_moments(self._h, C.byref(m)))
        return m

    def read_history(self):
        n = C.c_int64()
        _check("pic_read_history", lib().pic_read_history(self._h, None, 0, C.byref(n)))
        rows = (HistoryRow * max(n.value, 1))()
        _check("pic_read_history",
               lib().pic_read_history(self._h, C.cast(rows, C.c_void_p), n.value, C.byref(n)))
        return np.frombuffer(bytes(rows), dtype=HISTORY_DTYPE, count=n.value).copy()

    def read_particles(self, species):
        m = self.read_moments()
        n = m.n_minus if species == 0 else m.n_plus
        cell = np.zeros(n, np.int32); off = np.zeros(n); p = np.zeros(n)
        ids = np.zeros(n, np.uint64); n_out = C.c_int64()
        _check("pic_read_particles", lib().pic_read_particles(
            self._h, species, n, _ptr(cell), _ptr(off), _ptr(p), _ptr(ids), C.byref(n_out)))
        k = min(n, n_out.value)
        return {"cell": cell[:k], "off": off[:k], "p": p[:k], "id": ids[:k]}

    def read_photons(self):
        m = self.read_moments()
        n = m.photon_slots
        xq = np.zeros(n, np.int64); cs = np.zeros(n, np.int64); d = np.zeros(n, np.int32)
        ch = np.zeros(n, np.uint64); n_out = C.c_int64()
        _check("pic_read_photons", lib().pic_read_photons(
            self._h, n, _ptr(xq), _ptr(cs), _ptr(d), _ptr(ch), C.byref(n_out)))
        k = n_out.value
        return {"xq": xq[:k], "conv_step": cs[:k], "dir": d[:k], "child": ch[:k]}

    def set_fields(self, E):
        E = np.ascontiguousarray(E, np.float64)
        _check("pic_set_fields", lib().pic_set_fields(self._h, _ptr(E), self.n_cells))


class Gap(_GapView):
    """One gap over a torch-allocated device workspace (pic_create_gap)."""

    def __init__(self, params, device="cuda", stream=None, workspace=None):
        L = lib()
        st = L.pic_validate_params(C.byref(params))
        _check("pic_validate_params", st)
        nbytes = L.pic_workspace_bytes(C.byref(params))
        self.workspace = _device_workspace(nbytes, device, workspace)
        sh, self.stream = _stream_handle(stream)
        h = C.c_void_p()
        _check("pic_create_gap", L.pic_create_gap(C.byref(params), C.c_void_p(self.workspace.data_ptr()),
                                                  nbytes, sh, C.byref(h)))
        super().__init__(h, params, None)

    def prepare(self):
        """Sorts the seed and captures the step graphs now (pic_prepare)."""
        _check("pic_prepare", lib().pic_prepare(self._h))

    def step_n(self, n_steps, report=False):
        rep = StepReport() if report else None
        _check("pic_step_n", lib().pic_step_n(self._h, n_steps, C.byref(rep) if report else None))
        return rep

    def profile_push(self, enable=True):
        _check("pic_profile_push", lib().pic_profile_push(self._h, int(enable)))

    def read_push_time(self):
        ms, n = C.c_double(), C.c_int64()
        _check("pic_read_push_time", lib().pic_read_push_time(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def tuning(self):
        return _tuning("pic_tuning", self._h)

    def emission_split(self, max_push_chunks):
        """Steps whose plan holds fewer lepton chunks draw their emissions in the push."""
        _check("pic_emission_split", lib().pic_emission_split(self._h, int(max_push_chunks)))

    def close(self):
        """Frees the handle and drops this object's reference to the workspace."""
        if self._h:
            lib().pic_destroy(self._h)
            self._h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent gaps advanced by the same launches (pic_create_batch)."""

    def __init__(self, params_list, device="cuda", stream=None, workspace=None):
        L = lib()
        arr = (GapParams * len(params_list))(*params_list)
        nbytes = L.pic_batch_workspace_bytes(arr, len(params_list))
        if nbytes == 0:
            raise PicError("pic_batch_workspace_bytes", ERR_ARG)
        self.workspace = _device_workspace(nbytes, device, workspace)
        sh, self.stream = _stream_handle(stream)
        h = C.c_void_p()
        _check("pic_create_batch", L.pic_create_batch(arr, len(params_list),
                                                      C.c_void_p(self.workspace.data_ptr()),
                                                      nbytes, sh, C.byref(h)))
        self._h = h
        self._arr = arr
        self.gaps = [_GapView(L.pic_batch_gap(h, i), params_list[i], self)
                     for i in range(len(params_list))]

    def prepare(self):
        """Sorts the seeds and captures the step graphs now (pic_batch_prepare)."""
        _check("pic_batch_prepare", lib().pic_batch_prepare(self._h))

    def step_n(self, n_steps, statuses=False):
        out = np.zeros(len(self.gaps), np.int32) if statuses else None
        _check("pic_batch_step_n", lib().pic_batch_step_n(self._h, n_steps, _ptr(out)))
        return out

    def profile_push(self, enable=True):
        _check("pic_batch_profile_push", lib().pic_batch_profile_push(self._h, int(enable)))

    def read_push_time(self):
        ms, n = C.c_double(), C.c_int64()
        _check("pic_batch_read_push_time",
               lib().pic_batch_read_push_time(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def tuning(self):
        return _tuning("pic_batch_tuning", self._h)

    def emission_split(self, max_push_chunks):
        """Steps whose plan holds fewer lepton chunks draw their emissions in the push."""
        _check("pic_batch_emission_split", lib().pic_batch_emission_split(self._h, int(max_push_chunks)))

    def close(self):
        """Frees the handle and drops this object's reference to the workspace;
        the gap views of a closed batch must not be used."""
        if self._h:
            lib().pic_destroy_batch(self._h)
            self._h = None
        self.workspace = None
        self.gaps = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_plan(params_list, budget_bytes):
    arr = (GapParams * len(params_list))(*params_list)
    adm = np.zeros(len(params_list), np.uint8)
    ws = C.c_size_t()
    n = lib().pic_batch_plan(arr, len(params_list), budget_bytes, _ptr(adm), C.byref(ws))
    if n < 0:
        raise PicError("pic_batch_plan", n)
    return adm.astype(bool), ws.value
