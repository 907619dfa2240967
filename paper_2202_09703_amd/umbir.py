"""Python binding of libumbir.so (include/umbir.h): argument marshalling only.

Every computation runs in the HIP library; PyTorch supplies device memory and
the current stream.  The functions keep the C names without the prefix:
build_geometry, forward, adjoint, direct, sqs_denominator, reconstruct.
If the library has not been built, importing this module raises ImportError:
there is no fallback path.

Problem descriptions are duck-typed: any object with `medium` (speed,
thickness, atten, density), `grid` (nx, nz, dx, dz, x0, z0), `array` (tx_x,
rx_offset, beta) and `acq` (n_samples, fs, f_c, sigma_t, t_win, oversample)
attributes, in SI units, describes a problem.  A prior is any object with
p, q, T, sigma0, m, a and estimate_direct attributes.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

# torch goes first: it loads its own HIP runtime (SONAME libamdhip64.so.7), and
# the library's dependency on that SONAME then binds to the same copy, so one
# process never holds two HIP/HSA runtimes.
import torch  # noqa: E402,F401

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libumbir.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2202_09703_amd.build`")
_lib = C.CDLL(_LIB_PATH)

OK, EINVAL, ENOMEM, EDEVICE, ENOTSUP, EDIVERGED = 0, -1, -2, -3, -4, -5
STORAGE_F32, STORAGE_F16, STORAGE_BF16 = 0, 1, 2
TRACE_DTYPES = {STORAGE_F32: torch.float32, STORAGE_F16: torch.float16, STORAGE_BF16: torch.bfloat16}
WORK_FORWARD, WORK_ADJOINT, WORK_RECONSTRUCT = 0, 1, 2
BATCH_STREAMS, BATCH_GRAPH, BATCH_WORKLIST = 0, 1, 2
TABLE_DELAY, TABLE_APOD, TABLE_TAU, TABLE_BANK, TABLE_DBASIS, TABLE_OFFSET, TABLE_ATTEN = range(7)
MAX_LAYERS = 8

_dp = C.POINTER(C.c_double)


class _Medium(C.Structure):
    _fields_ = [("n_layers", C.c_int), ("speed", _dp), ("thickness", _dp), ("atten", _dp),
                ("density", _dp)]


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("nz", C.c_int), ("dx", C.c_double), ("dz", C.c_double),
                ("x0", C.c_double), ("z0", C.c_double)]


class _Array(C.Structure):
    _fields_ = [("n_scans", C.c_int), ("tx_x", _dp), ("n_rx", C.c_int), ("rx_offset", _dp),
                ("beta", C.c_int)]


class _Acq(C.Structure):
    _fields_ = [("n_samples", C.c_int), ("fs", C.c_double), ("f_c", C.c_double),
                ("sigma_t", C.c_double), ("t_win", C.c_double), ("oversample", C.c_int),
                ("storage", C.c_int), ("n_gamma", C.c_int)]


class _Problem(C.Structure):
    _fields_ = [("medium", _Medium), ("grid", _Grid), ("array", _Array), ("acq", _Acq)]


class _Prior(C.Structure):
    _fields_ = [("sigma", C.c_double), ("p", C.c_double), ("q", C.c_double), ("T", C.c_double),
                ("sigma0", C.c_double), ("m", C.c_double), ("a", C.c_double),
                ("estimate_direct", C.c_int)]


class _Dims(C.Structure):
    _fields_ = [("nx", C.c_int), ("nz", C.c_int), ("n_scans", C.c_int), ("n_rx", C.c_int),
                ("n_samples", C.c_int), ("n_off", C.c_int), ("window", C.c_int),
                ("oversample", C.c_int), ("n_layers", C.c_int), ("trace_groups", C.c_int),
                ("storage", C.c_int), ("n_gamma", C.c_int), ("gamma_step", C.c_double)]


class _Tuning(C.Structure):
    _fields_ = [("splat_blocks", C.c_int), ("gather_batch_kb", C.c_int), ("conv_grid", C.c_int),
                ("conv_tile_rows", C.c_int), ("corr_tile_rows", C.c_int), ("corr_blocks", C.c_int),
                ("operator_form", C.c_int), ("products", C.c_int), ("gather_form", C.c_int)]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class _KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_longlong), ("total_ms", C.c_double)]


_vp, _sz, _i = C.c_void_p, C.c_size_t, C.c_int
_SIGS = {
    "umbir_build_geometry": (_i, [C.POINTER(_Problem), _vp, C.POINTER(_vp)]),
    "umbir_geometry_free": (None, [_vp]),
    "umbir_geometry_bytes": (_sz, [_vp]),
    "umbir_estimate_bytes": (_sz, [C.POINTER(_Problem)]),
    "umbir_workspace_bytes": (_sz, [_vp, _i]),
    "umbir_forward": (_i, [_vp, _vp, _vp, _i, _vp, _sz, _vp]),
    "umbir_adjoint": (_i, [_vp, _vp, _vp, _vp, _sz, _vp]),
    "umbir_direct": (_i, [_vp, _vp, _vp, _i, _vp]),
    "umbir_sqs_denominator": (_i, [_vp, C.c_double, _vp, _vp, _sz, _vp]),
    "umbir_reconstruct": (_i, [_vp, C.POINTER(_Prior), _vp, _i, _vp, _vp, _vp, _vp, _sz, _vp]),
    "umbir_reconstruct_noalloc": (_i, [_vp, C.POINTER(_Prior), _vp, _i, _vp, _vp, _vp, _vp]),
    "umbir_reconstruct_icd": (_i, [_vp, C.POINTER(_Prior), _vp, _i, _i, _i, _vp, _vp, _vp, _vp, _sz, _vp]),
    "umbir_icd_workspace_bytes": (_sz, [_vp, _i, _i]),
    "umbir_get_dims": (_i, [_vp, C.POINTER(_Dims)]),
    "umbir_copy_table": (_i, [_vp, _i, _vp, _sz]),
    "umbir_get_tuning": (_i, [_vp, C.POINTER(_Tuning)]),
    "umbir_set_tuning": (_i, [_vp, C.POINTER(_Tuning)]),
    "umbir_autotune": (_i, [_vp, _vp, C.POINTER(_Tuning)]),
    "umbir_solver_bytes": (_sz, [_vp, _i]),
    "umbir_solver_create": (_i, [_vp, C.POINTER(_Prior), _vp, _vp, _vp, _i, _vp, C.POINTER(_vp)]),
    "umbir_solver_step": (_i, [_vp, _i, _vp]),
    "umbir_solver_iterations": (_i, [_vp]),
    "umbir_solver_read": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "umbir_solver_state_bytes": (_sz, [_vp]),
    "umbir_solver_free": (None, [_vp]),
    "umbir_batch_create": (_i, [C.POINTER(_vp), _i, _i, C.POINTER(_vp)]),
    "umbir_batch_step": (_i, [_vp, _i, _vp]),
    "umbir_batch_free": (None, [_vp]),
    "umbir_profile_enable": (None, [_i]),
    "umbir_profile_select": (None, [C.c_char_p]),
    "umbir_profile_stride": (None, [_i]),
    "umbir_profile_collect": (_i, [C.POINTER(_KernelTime), _i, C.POINTER(_i)]),
    "umbir_strerror": (C.c_char_p, [_i]),
    "umbir_last_error": (C.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTS = tuple(_SIGS)


class UmbirError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        detail = _lib.umbir_last_error().decode()
        super().__init__(f"{where}: {_lib.umbir_strerror(status).decode()} ({status}): {detail}")


def _check(status: int, where: str):
    if status != OK:
        raise UmbirError(status, where)


def _darr(values):
    vals = [float(v) for v in values]
    return (C.c_double * max(1, len(vals)))(*vals)


class Problem:
    """A ctypes umbir_problem built from a card-like object; keeps its arrays alive."""

    def __init__(self, card):
        med, g, a, q = card.medium, card.grid, card.array, card.acq
        n = len(med.speed)
        self._keep = [_darr(med.speed), _darr(med.thickness), _darr(med.atten or [0.0] * n),
                      _darr(med.density), _darr(a.tx_x), _darr(a.rx_offset)]
        sp, th, at, de, tx, rx = self._keep
        self.c = _Problem(
            _Medium(n, sp, th, at, de),
            _Grid(int(g.nx), int(g.nz), float(g.dx), float(g.dz), float(g.x0), float(g.z0)),
            _Array(len(a.tx_x), tx, len(a.rx_offset), rx, int(a.beta)),
            _Acq(int(q.n_samples), float(q.fs), float(q.f_c), float(q.sigma_t), float(q.t_win),
                 int(q.oversample), int(getattr(q, "storage", STORAGE_F32)), int(getattr(q, "n_gamma", 0))))


def estimate_bytes(card) -> int:
    return int(_lib.umbir_estimate_bytes(C.byref(Problem(card).c)))


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, name, shape=None, dtype=None):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


class Geometry:
    """Owns a built umbir_geometry (device tables resident until freed)."""

    def __init__(self, handle: C.c_void_p, device: int):
        self._h = handle
        self.device = device
        d = _Dims()
        _check(_lib.umbir_get_dims(self._h, C.byref(d)), "umbir_get_dims")
        self.nx, self.nz = d.nx, d.nz
        self.n_scans, self.n_rx, self.n_samples = d.n_scans, d.n_rx, d.n_samples
        self.n_off, self.window, self.oversample, self.n_layers = d.n_off, d.window, d.oversample, d.n_layers
        self.trace_groups = d.trace_groups
        self.storage = d.storage
        self.trace_dtype = TRACE_DTYPES[d.storage]
        self.n_gamma, self.gamma_step = d.n_gamma, d.gamma_step

    @property
    def handle(self):
        if not self._h:
            raise ValueError("geometry has been freed")
        return self._h

    @property
    def shape_key(self):
        """What the launch- and tile-shape tuning depends on (window L_h, record
        M, traces P x K, grid nz x nx, storage, and the rest of the shape)."""
        return (self.nx, self.nz, self.n_scans, self.n_rx, self.n_samples, self.oversample, self.window,
                self.n_layers, self.storage, self.n_gamma)

    def tuning(self) -> dict:
        t = _Tuning()
        _check(_lib.umbir_get_tuning(self.handle, C.byref(t)), "umbir_get_tuning")
        return t.as_dict()

    def set_tuning(self, splat_blocks: int = 0, gather_batch_kb: int = 0, conv_grid: int = 0,
                   conv_tile_rows: int = 0, corr_tile_rows: int = 0, corr_blocks: int = 0, operator_form: int = 0,
                   products: int = 0, gather_form: int = 0):
        """Launch and tile shapes, the operator's form, the matrix-core
        products and the gather's form (umbir_tuning); 0 keeps a field's
        value."""
        t = _Tuning(int(splat_blocks), int(gather_batch_kb), int(conv_grid), int(conv_tile_rows), int(corr_tile_rows),
                    int(corr_blocks), int(operator_form), int(products), int(gather_form))
        _check(_lib.umbir_set_tuning(self.handle, C.byref(t)), "umbir_set_tuning")

    def autotune(self, stream=None, cache: Optional[dict] = None) -> dict:
        """Time the tuning candidates on the device (umbir_autotune) and keep
        the fastest; with a cache, shapes seen before reuse their result."""
        key = self.shape_key
        if cache is not None and key in cache:
            self.set_tuning(**cache[key])
            return dict(cache[key])
        t = _Tuning()
        _check(_lib.umbir_autotune(self.handle, _stream(stream), C.byref(t)), "umbir_autotune")
        res = t.as_dict()
        if cache is not None:
            cache[key] = dict(res)
        return res

    @property
    def image_shape(self):
        return (self.nz, self.nx)

    @property
    def trace_shape(self):
        return (self.n_scans, self.n_rx, self.n_samples)

    @property
    def bytes(self) -> int:
        return int(_lib.umbir_geometry_bytes(self.handle))

    def workspace_bytes(self, kind: int) -> int:
        return int(_lib.umbir_workspace_bytes(self.handle, kind))

    def workspace(self, kind: int):
        import torch
        return torch.empty(self.workspace_bytes(kind), dtype=torch.uint8, device=f"cuda:{self.device}")

    def table(self, which: int) -> np.ndarray:
        P, K, M = self.trace_shape
        spec = {
            TABLE_DELAY: (np.int64, (self.nz, self.n_off)),
            TABLE_APOD: (np.float32, (self.nz, self.n_off)),
            TABLE_TAU: (np.float32, (self.nz,)),
            TABLE_BANK: (np.float32, (self.n_gamma, self.oversample * self.window + 2)),
            TABLE_DBASIS: (np.float32, (P, K, M)),
            TABLE_OFFSET: (np.int32, (P + P * K,)),
            TABLE_ATTEN: (np.float64, (self.nz, self.n_off)),
        }[which]
        out = np.empty(spec[1], dtype=spec[0])
        _check(_lib.umbir_copy_table(self.handle, which, out.ctypes.data_as(C.c_void_p), out.nbytes),
               "umbir_copy_table")
        return out

    def free(self):
        if self._h:
            _lib.umbir_geometry_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_geometry(card, stream=None) -> Geometry:
    import torch
    pb = Problem(card)
    h = C.c_void_p()
    _check(_lib.umbir_build_geometry(C.byref(pb.c), _stream(stream), C.byref(h)), "umbir_build_geometry")
    return Geometry(h, torch.cuda.current_device())


def _work(geom, work, kind):
    if work is None:
        work = geom.workspace(kind)
    return _ptr(work, "work"), C.c_size_t(work.numel() * work.element_size())


def forward(geom: Geometry, x, y=None, accumulate: bool = False, work=None, stream=None):
    """y = A x (or y += A x); x: [nz][nx] float32, y: [P][K][M] in the storage type."""
    import torch
    if y is None:
        y = torch.empty(geom.trace_shape, dtype=geom.trace_dtype, device=x.device)
    wp, wb = _work(geom, work, WORK_FORWARD)
    _check(_lib.umbir_forward(geom.handle, _ptr(x, "x", geom.image_shape, torch.float32),
                              _ptr(y, "y", geom.trace_shape, geom.trace_dtype), int(bool(accumulate)),
                              wp, wb, _stream(stream)), "umbir_forward")
    return y


def adjoint(geom: Geometry, r, x=None, work=None, stream=None):
    """x = A^T r; r: [P][K][M] in the storage type, x: [nz][nx] float32."""
    import torch
    if x is None:
        x = torch.empty(geom.image_shape, dtype=torch.float32, device=r.device)
    wp, wb = _work(geom, work, WORK_ADJOINT)
    _check(_lib.umbir_adjoint(geom.handle, _ptr(r, "r", geom.trace_shape, geom.trace_dtype),
                              _ptr(x, "x", geom.image_shape, torch.float32), wp, wb, _stream(stream)),
           "umbir_adjoint")
    return x


def direct(geom: Geometry, g, y=None, accumulate: bool = False, stream=None):
    """y = D g (or y += D g); g: [P][K] float32, y in the storage type."""
    import torch
    if y is None:
        y = torch.empty(geom.trace_shape, dtype=geom.trace_dtype, device=g.device)
    _check(_lib.umbir_direct(geom.handle, _ptr(g, "g", geom.trace_shape[:2], torch.float32),
                             _ptr(y, "y", geom.trace_shape, geom.trace_dtype), int(bool(accumulate)),
                             _stream(stream)), "umbir_direct")
    return y


def sqs_denominator(geom: Geometry, sigma: float, d=None, work=None, stream=None):
    """d = |A|^T |A| 1 / sigma^2 as [nz][nx] float32."""
    import torch
    dev = f"cuda:{geom.device}"
    if d is None:
        d = torch.empty(geom.image_shape, dtype=torch.float32, device=dev)
    wp, wb = _work(geom, work, WORK_RECONSTRUCT)
    _check(_lib.umbir_sqs_denominator(geom.handle, float(sigma), _ptr(d, "d", geom.image_shape, torch.float32),
                                      wp, wb, _stream(stream)), "umbir_sqs_denominator")
    return d


def make_prior(prior, sigma: float) -> _Prior:
    return _Prior(float(sigma), float(prior.p), float(prior.q), float(prior.T), float(prior.sigma0),
                  float(prior.m), float(prior.a), int(bool(prior.estimate_direct)))


def reconstruct(geom: Geometry, prior, sigma: float, y, n_iter: int, x=None, g=None, cost=None,
                work=None, stream=None):
    """MAP reconstruction (Eq. (18)); returns (x, g, cost) as device tensors.

    x, g: warm start (zeros if None), updated in place; cost: float64 of
    n_iter + 1 entries (allocated if None)."""
    import torch
    dev = y.device
    if x is None:
        x = torch.zeros(geom.image_shape, dtype=torch.float32, device=dev)
    if g is None:
        g = torch.zeros(geom.trace_shape[:2], dtype=torch.float32, device=dev)
    if cost is None:
        cost = torch.empty(n_iter + 1, dtype=torch.float64, device=dev)
    pr = make_prior(prior, sigma)
    wp, wb = _work(geom, work, WORK_RECONSTRUCT)
    _check(_lib.umbir_reconstruct(geom.handle, C.byref(pr), _ptr(y, "y", geom.trace_shape, geom.trace_dtype),
                                  int(n_iter), _ptr(x, "x", geom.image_shape, torch.float32),
                                  _ptr(g, "g", geom.trace_shape[:2], torch.float32),
                                  _ptr(cost, "cost", (n_iter + 1,), torch.float64), wp, wb,
                                  _stream(stream)), "umbir_reconstruct")
    return x, g, cost


NOALLOC_SCRATCH_BYTES = 160 << 20  # UMBIR_NOALLOC_SCRATCH_MIB


def reconstruct_noalloc(geom: Geometry, prior, sigma: float, y, n_iter: int, x, g, cost, stream=None):
    """umbir_reconstruct_noalloc: as reconstruct, with the library's static
    device scratch as workspace; x, g (warm start, updated in place) and cost
    (float64, n_iter + 1 entries) are the caller's tensors (the call itself
    allocates nothing)."""
    import torch
    pr = make_prior(prior, sigma)
    _check(_lib.umbir_reconstruct_noalloc(geom.handle, C.byref(pr),
                                          _ptr(y, "y", geom.trace_shape, geom.trace_dtype), int(n_iter),
                                          _ptr(x, "x", geom.image_shape, torch.float32),
                                          _ptr(g, "g", geom.trace_shape[:2], torch.float32),
                                          _ptr(cost, "cost", (n_iter + 1,), torch.float64),
                                          _stream(stream)), "umbir_reconstruct_noalloc")
    return x, g, cost


def reconstruct_icd(geom: Geometry, prior, sigma: float, y, n_sweeps: int, group=(8, 8), x=None, g=None,
                    cost=None, stream=None):
    """MAP reconstruction (Eq. (18)) by ICD over a group_rows x group_cols
    lattice of voxel groups; returns (x, g, cost) as device tensors (cost:
    float64, n_sweeps + 1 entries).  x, g: warm start, updated in place."""
    import torch
    dev = y.device
    if x is None:
        x = torch.zeros(geom.image_shape, dtype=torch.float32, device=dev)
    if g is None:
        g = torch.zeros(geom.trace_shape[:2], dtype=torch.float32, device=dev)
    if cost is None:
        cost = torch.empty(n_sweeps + 1, dtype=torch.float64, device=dev)
    pr = make_prior(prior, sigma)
    rows, cols = int(group[0]), int(group[1])
    _check(_lib.umbir_reconstruct_icd(geom.handle, C.byref(pr), _ptr(y, "y", geom.trace_shape, geom.trace_dtype),
                                      int(n_sweeps), rows, cols, _ptr(x, "x", geom.image_shape, torch.float32),
                                      _ptr(g, "g", geom.trace_shape[:2], torch.float32),
                                      _ptr(cost, "cost", (n_sweeps + 1,), torch.float64), None, 0,
                                      _stream(stream)), "umbir_reconstruct_icd")
    return x, g, cost


def icd_workspace_bytes(geom: Geometry, group=(8, 8)) -> int:
    return int(_lib.umbir_icd_workspace_bytes(geom.handle, int(group[0]), int(group[1])))


class Solver:
    """Resident MAP solver session (umbir_solver_*): state, curvature and one
    captured graph per iteration live on the device until free()."""

    def __init__(self, geom: Geometry, prior, sigma: float, y, max_iter: int, x0=None, g0=None, stream=None):
        import torch
        self.geom = geom
        self.max_iter = int(max_iter)
        pr = make_prior(prior, sigma)
        h = C.c_void_p()
        _check(_lib.umbir_solver_create(geom.handle, C.byref(pr), _ptr(y, "y", geom.trace_shape, geom.trace_dtype),
                                        _ptr(x0, "x0", geom.image_shape, torch.float32),
                                        _ptr(g0, "g0", geom.trace_shape[:2], torch.float32), self.max_iter,
                                        _stream(stream), C.byref(h)), "umbir_solver_create")
        self._h = h
        self.device = y.device

    @property
    def handle(self):
        if not self._h:
            raise ValueError("solver has been freed")
        return self._h

    @property
    def iterations(self) -> int:
        return int(_lib.umbir_solver_iterations(self.handle))

    @property
    def bytes(self) -> int:
        return int(_lib.umbir_solver_state_bytes(self.handle))

    def step(self, n_iter: int, stream=None):
        _check(_lib.umbir_solver_step(self.handle, int(n_iter), _stream(stream)), "umbir_solver_step")

    def read(self, x=None, g=None, with_cost: bool = True, stream=None):
        """Queues copies of (x, g) and the cost history; returns device tensors."""
        import torch
        geom = self.geom
        if x is None:
            x = torch.empty(geom.image_shape, dtype=torch.float32, device=self.device)
        if g is None:
            g = torch.empty(geom.trace_shape[:2], dtype=torch.float32, device=self.device)
        cost = torch.empty(self.iterations + 1, dtype=torch.float64, device=self.device) if with_cost else None
        _check(_lib.umbir_solver_read(self.handle, _ptr(x, "x", geom.image_shape, torch.float32),
                                      _ptr(g, "g", geom.trace_shape[:2], torch.float32),
                                      _ptr(cost, "cost", None, torch.float64) if cost is not None else None,
                                      _stream(stream)), "umbir_solver_read")
        return x, g, cost

    def free(self):
        if self._h:
            _lib.umbir_solver_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Batch:
    """Many resident sessions advanced together (umbir_batch_*): one graph
    launch runs one iteration of every session, side by side on the device."""

    def __init__(self, sessions, mode: int = 0):
        self.sessions = list(sessions)
        arr = (C.c_void_p * len(self.sessions))(*[s.handle.value for s in self.sessions])
        h = C.c_void_p()
        _check(_lib.umbir_batch_create(arr, len(self.sessions), int(mode), C.byref(h)), "umbir_batch_create")
        self._h = h

    @property
    def handle(self):
        if not self._h:
            raise ValueError("batch has been freed")
        return self._h

    def step(self, n_iter: int, stream=None):
        _check(_lib.umbir_batch_step(self.handle, int(n_iter), _stream(stream)), "umbir_batch_step")

    def free(self):
        if self._h:
            _lib.umbir_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def solver_bytes(geom: Geometry, max_iter: int) -> int:
    return int(_lib.umbir_solver_bytes(geom.handle, int(max_iter)))


def profile_enable(on: bool = True):
    """Turn per-kernel event timing on or off (process-wide)."""
    _lib.umbir_profile_enable(int(bool(on)))


def profile_select(names=None):
    """Time only the kernels named (an iterable of names, or None for all)."""
    _lib.umbir_profile_select(",".join(names).encode() if names else None)


def profile_stride(every: int = 1):
    """With a selection set, time only every `every`-th launch of each selected kernel."""
    _lib.umbir_profile_stride(int(every))


def profile_collect() -> dict:
    """{kernel name: (launches, total ms)} since the last collect; resets the totals."""
    buf = (_KernelTime * 64)()
    n = C.c_int()
    _check(_lib.umbir_profile_collect(buf, 64, C.byref(n)), "umbir_profile_collect")
    return {buf[k].name.decode(): (int(buf[k].launches), float(buf[k].total_ms)) for k in range(min(n.value, 64))}


def library_path() -> str:
    return _LIB_PATH
