"""MI355X (gfx950) Local Exponential Method: Python binding of ``liblem.so``.

A thin ctypes layer over the C ABI in ``include/lem.h``: it marshals
arguments (device pointers of torch tensors, HIP stream handles, host numpy
arrays) and returns results; every step of the method runs in the library's
HIP kernels.  There is no fallback: if the library is missing, importing the
binding's entry points raises.

The Local Exponential Method (L. Bonaventura, section 3) advances du/dt = A u
on overlapping subdomains: each region (core + buffer) is advanced by its own
local exponential exp(dt A_M) and the core rows overwrite the global state.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblem.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lem.h")

LEM_OK = 0
STATUS_NAMES = {0: "LEM_OK", 1: "LEM_ERR_INVALID", 2: "LEM_ERR_NOMEM", 3: "LEM_ERR_HIP",
                4: "LEM_ERR_NOT_CONVERGED", 5: "LEM_ERR_BUDGET", 6: "LEM_ERR_UNSUPPORTED",
                7: "LEM_ERR_NOT_FOUND", 8: "LEM_ERR_NONFINITE"}
METHODS = {"krylov": 0, "dense": 1, "global": 2, "kronecker": 4}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x2": 2, "bf16x3": 3}


class LemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Operator(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int32), ("dx", ctypes.c_double),
                ("vel", ctypes.c_double * 2), ("nu", ctypes.c_double),
                ("nu_field", ctypes.POINTER(ctypes.c_double)),
                ("forcing", ctypes.POINTER(ctypes.c_double)),
                ("vel_faces", ctypes.POINTER(ctypes.c_double)), ("dy", ctypes.c_double)]


class _Options(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("n_states", ctypes.c_int32), ("core", ctypes.c_int32),
                ("halo", ctypes.c_int32), ("halo_min", ctypes.c_int32),
                ("halo_max", ctypes.c_int32), ("halo_tol", ctypes.c_double),
                ("krylov_m", ctypes.c_int32), ("krylov_m_max", ctypes.c_int32),
                ("max_substeps", ctypes.c_int32), ("krylov_tol", ctypes.c_double),
                ("use_graph", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("dry_run", ctypes.c_int32), ("expm", ctypes.c_int32),
                ("columns", ctypes.c_int32), ("core_max", ctypes.c_int32),
                ("tile", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int32), ("n_unique", ctypes.c_int32),
                ("n_loc_total", ctypes.c_int64), ("n_loc_max", ctypes.c_int32),
                ("halo_min", ctypes.c_int32), ("halo_max", ctypes.c_int32),
                ("halo_clamped", ctypes.c_int32), ("m_min", ctypes.c_int32),
                ("m_max", ctypes.c_int32), ("substeps_max", ctypes.c_int32),
                ("squarings", ctypes.c_int32), ("bytes_blocks", ctypes.c_int64),
                ("bytes_work", ctypes.c_int64), ("device_status", ctypes.c_int32),
                ("max_estimate", ctypes.c_double), ("plan_ms", ctypes.c_double),
                ("tile_config", ctypes.c_int32), ("krylov_bytes_step", ctypes.c_double),
                ("krylov_bytes_streamed", ctypes.c_double), ("resident_steps", ctypes.c_int32)]


_lib = None


def load() -> ctypes.CDLL:
    """Load liblem.so (built in-tree by ``build.py``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_1505_02248_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, D, VP = ctypes.POINTER, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
    lib.lem_options_default.argtypes = [P(_Options)]
    lib.lem_options_default.restype = None
    lib.lem_plan.argtypes = [P(_Operator), D, P(_Options), VP, P(VP)]
    lib.lem_step.argtypes = [VP, VP, VP, I32, VP]
    lib.lem_global_expmv.argtypes = [P(_Operator), D, VP, VP, I32, D, I32, VP]
    lib.lem_global_expmv_static.argtypes = [P(_Operator), D, VP, VP, I32, D, I32, VP]
    lib.lem_ere_plan.argtypes = [P(_Burgers), D, I32, I32, I32, I32, VP, P(VP)]
    lib.lem_schrodinger_plan.argtypes = [P(_Schrodinger), D, I32, I32, I32, I32, VP, P(VP)]
    lib.lem_plan_query.argtypes = [VP, P(_Info)]
    lib.lem_plan_copy_maps.argtypes = [VP, P(I32), P(I32), P(I32)]
    lib.lem_plan_copy_krylov.argtypes = [VP, P(I32), P(I32)]
    lib.lem_plan_copy_block.argtypes = [VP, I32, P(D), P(I32), P(I32)]
    lib.lem_plan_destroy.argtypes = [VP]
    lib.lem_last_error.restype = ctypes.c_char_p
    for name in ("lem_plan", "lem_step", "lem_global_expmv", "lem_global_expmv_static",
                 "lem_plan_query",
                 "lem_plan_copy_maps", "lem_plan_copy_krylov", "lem_plan_copy_block",
                 "lem_plan_destroy"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def declared_functions(header: str = HEADER):
    """Names of the functions declared in include/lem.h."""
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    pat = r"^\s*(?:lem_status|void|const\s+char\s*\*)\s*(lem_[a-z_0-9]+)\s*\("
    return sorted(set(re.findall(pat, text, flags=re.M)))


def _check(status: int) -> None:
    if status != LEM_OK:
        raise LemError(status, load().lem_last_error().decode())


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


class Operator:
    """Periodic advection-diffusion operator of the model problem (eq. (2)),
    centered finite differences on n (1D) or n x n (2D) points.  ``vel_faces``
    (shape (ndim, ny, n), replacing ``vel``) gives face velocities for the
    conservative form of eq. ibv2d; ``dy`` the y spacing of an anisotropic
    mesh (None: dx)."""

    def __init__(self, ndim: int, n: int, dx: float, vel=(1.0, 0.0), nu: float = 0.0,
                 nu_field: Optional[np.ndarray] = None, forcing: Optional[np.ndarray] = None,
                 vel_faces: Optional[np.ndarray] = None, dy: Optional[float] = None):
        self.ndim, self.n, self.dx = int(ndim), int(n), float(dx)
        self.vel = (float(vel[0]), float(vel[1]) if len(vel) > 1 else 0.0)
        self.nu = float(nu)
        self.nu_field = None if nu_field is None else np.ascontiguousarray(nu_field, dtype=np.float64).reshape(-1)
        # source g of du/dt = A u + g (rate units), shape (N,) or (N, n_states)
        self.forcing = None if forcing is None else np.ascontiguousarray(forcing, dtype=np.float64)
        self.vel_faces = (None if vel_faces is None
                          else np.ascontiguousarray(vel_faces, dtype=np.float64).reshape(-1))
        self.dy = 0.0 if dy is None else float(dy)

    @property
    def N(self) -> int:
        return self.n ** self.ndim

    @classmethod
    def from_problem(cls, p) -> "Operator":
        return cls(p.ndim, p.n, p.dx, p.vel, p.nu if p.nu is not None else 0.0, p.nu_field,
                   vel_faces=getattr(p, "vel_faces", None), dy=getattr(p, "dy", None))

    def _c(self) -> _Operator:
        o = _Operator()
        o.ndim, o.n, o.dx = self.ndim, self.n, self.dx
        o.vel[0], o.vel[1] = self.vel
        o.nu = self.nu
        if self.nu_field is not None:
            if self.nu_field.size != self.N:
                raise ValueError("nu_field must have N entries")
            o.nu_field = self.nu_field.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            o.nu_field = None
        if self.forcing is not None:
            if self.forcing.shape[0] != self.N:
                raise ValueError("forcing must have N rows")
            o.forcing = self.forcing.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            o.forcing = None
        if self.vel_faces is not None:
            if self.vel_faces.size != self.ndim * self.N:
                raise ValueError("vel_faces must have ndim x N entries")
            o.vel_faces = self.vel_faces.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            o.vel_faces = None
        o.dy = self.dy
        return o


def _tensor_ptr(t, N: int, ns: int) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError("state must be a float64 CUDA (HIP) tensor")
    if not t.is_contiguous() or t.numel() != N * ns:
        raise ValueError(f"state must be contiguous with {N * ns} elements")
    return t.data_ptr()


class Plan:
    """A planned LEM stepper (``lem_plan``); see include/lem.h."""

    def __init__(self, op: Operator, dt: float, method: str = "krylov",
                 precision: str = "fp64", n_states: int = 1, core: int = 0,
                 halo: int = 0, halo_min: int = 4, halo_max: int = 64,
                 halo_tol: float = 1e-8, krylov_m: int = 0, krylov_m_max: int = 30,
                 max_substeps: int = 64, krylov_tol: float = 1e-13,
                 use_graph: bool = False, autotune: bool = False, dry_run: bool = False,
                 columns: bool = False, expm: str = "pade", tile: int = -1, core_max: int = 0,
                 stream=None):
        lib = load()
        o = _Options()
        lib.lem_options_default(ctypes.byref(o))
        o.method = METHODS[method]
        o.precision = PRECISIONS[precision]
        o.n_states, o.core, o.halo = n_states, core, halo
        o.halo_min, o.halo_max, o.halo_tol = halo_min, halo_max, halo_tol
        o.krylov_m, o.krylov_m_max, o.max_substeps = krylov_m, krylov_m_max, max_substeps
        o.krylov_tol = krylov_tol
        o.use_graph, o.autotune, o.dry_run = int(use_graph), int(autotune), int(dry_run)
        o.columns = int(columns)
        o.tile = int(tile)
        o.core_max = int(core_max)
        o.expm = {"pade": 0, "taylor": 1}[expm]
        self.op, self.dt, self.n_states, self.method = op, float(dt), int(n_states), method
        if op.forcing is not None and op.forcing.size != op.N * int(n_states):
            raise ValueError("forcing must hold N x n_states values")
        self._op_c = op._c()
        h = ctypes.c_void_p()
        st = 0 if dry_run else _stream_handle(stream)
        _check(lib.lem_plan(ctypes.byref(self._op_c), self.dt, ctypes.byref(o),
                            ctypes.c_void_p(st), ctypes.byref(h)))
        self._h = h

    def step(self, x_in, x_out, n_steps: int = 1, stream=None) -> None:
        N, ns = self.op.N, self.n_states
        _check(load().lem_step(self._h, ctypes.c_void_p(_tensor_ptr(x_in, N, ns)),
                               ctypes.c_void_p(_tensor_ptr(x_out, N, ns)), int(n_steps),
                               ctypes.c_void_p(_stream_handle(stream))))

    def query(self) -> dict:
        info = _Info()
        _check(load().lem_plan_query(self._h, ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in _Info._fields_}

    def maps(self):
        """(boxes [nb, 5], gather [sum n_loc], scatter [N]) as int32 arrays."""
        q = self.query()
        boxes = np.zeros((q["n_blocks"], 5), dtype=np.int32)
        gather = np.zeros(q["n_loc_total"], dtype=np.int32)
        scatter = np.zeros(self.op.N, dtype=np.int32)
        P = ctypes.POINTER(ctypes.c_int32)
        _check(load().lem_plan_copy_maps(self._h, boxes.ctypes.data_as(P),
                                         gather.ctypes.data_as(P), scatter.ctypes.data_as(P)))
        return boxes, gather, scatter

    def krylov(self):
        nb = max(self.query()["n_blocks"], 1)
        m = np.zeros(nb, dtype=np.int32)
        s = np.zeros(nb, dtype=np.int32)
        P = ctypes.POINTER(ctypes.c_int32)
        _check(load().lem_plan_copy_krylov(self._h, m.ctypes.data_as(P), s.ctypes.data_as(P)))
        return m, s

    def block(self, unique: int = 0) -> np.ndarray:
        r, c = ctypes.c_int32(), ctypes.c_int32()
        _check(load().lem_plan_copy_block(self._h, unique, None, ctypes.byref(r), ctypes.byref(c)))
        out = np.zeros((r.value, c.value), dtype=np.float64)
        _check(load().lem_plan_copy_block(self._h, unique,
                                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          None, None))
        return out

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            load().lem_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Burgers(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("dx", ctypes.c_double), ("nu", ctypes.c_double)]


class _Schrodinger(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("L", ctypes.c_double), ("kappa", ctypes.c_double)]


class _Grid1D:
    def __init__(self, n: int):
        self.N = int(n)


class ErePlan(Plan):
    """Exponential Rosenbrock-Euler LEM steps for periodic viscous Burgers
    (``lem_ere_plan``); step/query/maps as for ``Plan``."""

    def __init__(self, n: int, dx: float, nu: float, dt: float, n_states: int = 1,
                 core: int = 50, halo: int = 15, refresh: int = 5, stream=None):
        lib = load()
        b = _Burgers()
        b.n, b.dx, b.nu = int(n), float(dx), float(nu)
        self.op, self.dt, self.n_states, self.method = _Grid1D(n), float(dt), int(n_states), "rosenbrock"
        h = ctypes.c_void_p()
        _check(lib.lem_ere_plan(ctypes.byref(b), self.dt, int(n_states), int(core), int(halo),
                                int(refresh), ctypes.c_void_p(_stream_handle(stream)),
                                ctypes.byref(h)))
        self._h = h


class SchrodingerPlan(Plan):
    """LEM steps of the 1D Schroedinger equation with a harmonic potential
    (``lem_schrodinger_plan``).  States are real tensors of shape
    (2 n, n_states) holding the complex field interleaved per node (real
    part at row 2 j, imaginary part at row 2 j + 1); ``to_real_form`` and
    ``from_real_form`` convert from and to complex (n, n_states) tensors.
    ``query``/``maps`` report the doubled grid of 2 n real unknowns."""

    def __init__(self, n: int, L: float, kappa: float, dt: float, n_states: int = 1,
                 core: int = 100, halo: int = 20, autotune: bool = False, stream=None):
        lib = load()
        o = _Schrodinger()
        o.n, o.L, o.kappa = int(n), float(L), float(kappa)
        self.n = int(n)
        self.op, self.dt, self.n_states, self.method = _Grid1D(2 * n), float(dt), int(n_states), "dense"
        h = ctypes.c_void_p()
        _check(lib.lem_schrodinger_plan(ctypes.byref(o), self.dt, int(n_states), int(core),
                                        int(halo), 1 if autotune else 0,
                                        ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(h)))
        self._h = h

    @staticmethod
    def to_real_form(c):
        """complex (n, ns) torch tensor -> float64 (2 n, ns), interleaved per node."""
        import torch
        n, ns = c.shape
        return torch.view_as_real(c.to(torch.complex128)).permute(0, 2, 1).contiguous().reshape(2 * n, ns)

    @staticmethod
    def from_real_form(x):
        """float64 (2 n, ns) interleaved per node -> complex128 (n, ns)."""
        import torch
        n2, ns = x.shape
        return torch.view_as_complex(x.reshape(n2 // 2, 2, ns).permute(0, 2, 1).contiguous())


def global_expmv(op: Operator, t: float, x, y, n_states: int = 1, tol: float = 1e-13,
                 m_max: int = 40, stream=None) -> None:
    """y = exp(t A) x (+ phi_1(t A)(t g) with a forcing) on the whole grid
    (``lem_global_expmv``)."""
    N = op.N
    if op.forcing is not None and op.forcing.size != N * int(n_states):
        raise ValueError("forcing must hold N x n_states values")
    oc = op._c()
    _check(load().lem_global_expmv(ctypes.byref(oc), float(t),
                                   ctypes.c_void_p(_tensor_ptr(x, N, n_states)),
                                   ctypes.c_void_p(_tensor_ptr(y, N, n_states)), int(n_states),
                                   float(tol), int(m_max), ctypes.c_void_p(_stream_handle(stream))))


def global_expmv_static(op: Operator, t: float, x, y, n_states: int = 1, tol: float = 1e-13,
                        m_max: int = 40, stream=None) -> None:
    """As ``global_expmv`` but with no device allocation: the work space comes
    from the library's static per-device scratch (``lem_global_expmv_static``)."""
    N = op.N
    if op.forcing is not None and op.forcing.size != N * int(n_states):
        raise ValueError("forcing must hold N x n_states values")
    oc = op._c()
    _check(load().lem_global_expmv_static(ctypes.byref(oc), float(t),
                                          ctypes.c_void_p(_tensor_ptr(x, N, n_states)),
                                          ctypes.c_void_p(_tensor_ptr(y, N, n_states)),
                                          int(n_states), float(tol), int(m_max),
                                          ctypes.c_void_p(_stream_handle(stream))))


# ------------------------------------------------------------------ serving --

REQ_STATES = {0: "queued", 1: "active", 2: "done", 3: "failed"}


class _ServerOptions(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_active", ctypes.c_int32),
                ("halo_tol", ctypes.c_double), ("halo_min", ctypes.c_int32),
                ("halo_max", ctypes.c_int32), ("max_overhead", ctypes.c_double),
                ("krylov_tol", ctypes.c_double), ("krylov_m_max", ctypes.c_int32),
                ("max_substeps", ctypes.c_int32), ("dry_run", ctypes.c_int32),
                ("steps_per_tick", ctypes.c_int32)]


class _RequestInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("method", ctypes.c_int32), ("core", ctypes.c_int32),
                ("halo", ctypes.c_int32), ("n_blocks", ctypes.c_int32), ("m_max", ctypes.c_int32),
                ("substeps_max", ctypes.c_int32), ("n_steps", ctypes.c_int32),
                ("steps_done", ctypes.c_int32), ("bytes", ctypes.c_int64),
                ("t_submit_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double),
                ("t_done_ms", ctypes.c_double), ("error", ctypes.c_int32)]


class _ServerInfo(ctypes.Structure):
    _fields_ = [("n_queued", ctypes.c_int32), ("n_active", ctypes.c_int32),
                ("n_done", ctypes.c_int32), ("n_failed", ctypes.c_int32),
                ("ticks", ctypes.c_int64), ("bytes_in_use", ctypes.c_int64),
                ("bytes_budget", ctypes.c_int64), ("dof_steps", ctypes.c_double),
                ("device_status", ctypes.c_int32)]


def _server_lib():
    lib = load()
    if getattr(lib, "_server_ready", False):
        return lib
    P, VP = ctypes.POINTER, ctypes.c_void_p
    lib.lem_server_options_default.argtypes = [P(_ServerOptions)]
    lib.lem_server_options_default.restype = None
    lib.lem_server_create.argtypes = [P(_ServerOptions), VP, P(VP)]
    lib.lem_server_submit.argtypes = [VP, P(_Operator), ctypes.c_double, ctypes.c_int32,
                                      P(ctypes.c_double), P(ctypes.c_uint64)]
    lib.lem_server_tick.argtypes = [VP, P(ctypes.c_int32), P(ctypes.c_int32)]
    lib.lem_server_poll.argtypes = [VP, ctypes.c_uint64, P(ctypes.c_int32)]
    lib.lem_server_request_info.argtypes = [VP, ctypes.c_uint64, P(_RequestInfo)]
    lib.lem_server_fetch.argtypes = [VP, ctypes.c_uint64, P(ctypes.c_double)]
    lib.lem_server_query.argtypes = [VP, P(_ServerInfo)]
    lib.lem_server_destroy.argtypes = [VP]
    for name in ("lem_server_create", "lem_server_submit", "lem_server_tick", "lem_server_poll",
                 "lem_server_request_info", "lem_server_fetch", "lem_server_query",
                 "lem_server_destroy"):
        getattr(lib, name).restype = ctypes.c_int
    lib._server_ready = True
    return lib


class Server:
    """Continuous-batching LEM server (``lem_server_*``); see include/lem.h."""

    def __init__(self, hbm_budget: int = 8 << 30, max_active: int = 256,
                 halo_tol: float = 1e-8, halo_min: int = 4, halo_max: int = 56,
                 max_overhead: float = 4.0, krylov_tol: float = 1e-12,
                 krylov_m_max: int = 30, max_substeps: int = 64, dry_run: bool = False,
                 steps_per_tick: int = 1, stream=None):
        lib = _server_lib()
        o = _ServerOptions()
        lib.lem_server_options_default(ctypes.byref(o))
        o.hbm_budget, o.max_active = int(hbm_budget), int(max_active)
        o.halo_tol, o.halo_min, o.halo_max = halo_tol, halo_min, halo_max
        o.max_overhead, o.krylov_tol = max_overhead, krylov_tol
        o.krylov_m_max, o.max_substeps, o.dry_run = krylov_m_max, max_substeps, int(dry_run)
        o.steps_per_tick = int(steps_per_tick)
        h = ctypes.c_void_p()
        st = 0 if dry_run else _stream_handle(stream)
        _check(lib.lem_server_create(ctypes.byref(o), ctypes.c_void_p(st), ctypes.byref(h)))
        self._h = h
        self._sizes = {}

    def submit(self, op: Operator, dt: float, n_steps: int, x0: np.ndarray) -> int:
        x0 = np.ascontiguousarray(x0, dtype=np.float64).reshape(-1)
        if x0.size != op.N:
            raise ValueError("x0 must have N entries")
        oc = op._c()
        rid = ctypes.c_uint64()
        _check(_server_lib().lem_server_submit(self._h, ctypes.byref(oc), float(dt), int(n_steps),
                                               x0.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                               ctypes.byref(rid)))
        self._sizes[rid.value] = op.N
        return rid.value

    def tick(self):
        a, q = ctypes.c_int32(), ctypes.c_int32()
        _check(_server_lib().lem_server_tick(self._h, ctypes.byref(a), ctypes.byref(q)))
        return a.value, q.value

    def poll(self, rid: int) -> str:
        st = ctypes.c_int32()
        _check(_server_lib().lem_server_poll(self._h, rid, ctypes.byref(st)))
        return REQ_STATES[st.value]

    def request_info(self, rid: int) -> dict:
        info = _RequestInfo()
        _check(_server_lib().lem_server_request_info(self._h, rid, ctypes.byref(info)))
        d = {f: getattr(info, f) for f, _ in _RequestInfo._fields_}
        d["state"] = REQ_STATES[d["state"]]
        d["method"] = {v: k for k, v in METHODS.items()}[d["method"]]
        return d

    def fetch(self, rid: int) -> np.ndarray:
        out = np.empty(self._sizes[rid], dtype=np.float64)
        _check(_server_lib().lem_server_fetch(self._h, rid,
                                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        self._sizes.pop(rid, None)
        return out

    def query(self) -> dict:
        info = _ServerInfo()
        _check(_server_lib().lem_server_query(self._h, ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in _ServerInfo._fields_}

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            _server_lib().lem_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
