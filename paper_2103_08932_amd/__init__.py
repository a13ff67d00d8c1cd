"""MI355X (gfx950) splitting random-choice dynamic relaxation for total Lagrangian SPH.

A thin ctypes binding of ``libtlsph_dr.so`` (declared in ``include/tlsph_dr.h``).  Every step of
the relaxation runs in the library's HIP kernels; this module only marshals arguments.  PyTorch
supplies device memory (through the caching allocator) and the HIP stream.  If the library has
not been built the import of this package still succeeds, but every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# TLSPH_LIB selects another build of the same library (for example one compiled with different
# tuning constants); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("TLSPH_LIB") or os.path.join(HERE, "libtlsph_dr.so")

OK, NOT_CONVERGED = 0, 1
E_INVALID, E_NOMEM, E_SINGULAR_B0, E_CELL_ADJ, E_NONFINITE, E_DIVERGED, E_DEVICE, E_LIMIT = -1, -2, -3, -4, -5, -6, -7, -8
FP32, FP64 = 32, 64
SVK, NEOHOOKE = 0, 1
MODELS = {"svk": SVK, "nh": NEOHOOKE, "neohooke": NEOHOOKE}
PAIRWISE, PARTICLE = 0, 1
SCHEMES = {"pairwise": PAIRWISE, "particle": PARTICLE}
PASS_NAMES = ("drift", "passA", "passB", "passD", "passC", "finish")

_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class _Allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", C.c_void_p)]


class _BodyDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int64), ("X0", C.POINTER(C.c_double)), ("clamped", C.POINTER(C.c_uint8)),
                ("dp", C.c_double), ("h_over_dp", C.c_double), ("rho0", C.c_double), ("precision", C.c_int),
                ("stream", C.c_void_p), ("alloc", _Allocator)]


class _Report(C.Structure):
    _fields_ = [("steps", C.c_int64), ("damped_steps", C.c_int64), ("step_index", C.c_int64),
                ("residual", C.c_double), ("kinetic_energy", C.c_double), ("force_residual", C.c_double),
                ("dt", C.c_double), ("wall_s", C.c_double), ("window", C.c_int64), ("converged", C.c_int)]


class _Request(C.Structure):
    _fields_ = [("body", _BodyDesc), ("model", C.c_int), ("E", C.c_double), ("nu", C.c_double),
                ("g", C.c_double * 3), ("accel", C.POINTER(C.c_double)), ("eta", C.c_double), ("beta", C.c_double),
                ("Lc", C.c_double), ("alpha", C.c_double), ("seed", C.c_uint64), ("tol", C.c_double),
                ("max_steps", C.c_int64), ("scheme", C.c_int)]


class _ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64), ("pending", C.c_int64),
                ("in_setup", C.c_int64), ("active", C.c_int64), ("peak_active", C.c_int64), ("chunks", C.c_int64),
                ("batch_steps", C.c_int64), ("pool_bytes", C.c_size_t), ("pool_used", C.c_size_t),
                ("pool_peak", C.c_size_t)]


class TLSPHError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tlsph error {code}: {msg}")
        self.code = code


_lib = None
_dp = C.POINTER(C.c_double)


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2103_08932_amd.build.build() "
                               "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        L.tlsph_last_error.restype = C.c_char_p
        L.tlsph_version.restype = C.c_char_p
        L.tlsph_create_body.argtypes = [C.POINTER(_BodyDesc), C.POINTER(C.c_void_p)]
        L.tlsph_set_material.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double]
        L.tlsph_set_loads.argtypes = [C.c_void_p, _dp, _dp]
        L.tlsph_set_damping.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_uint64]
        L.tlsph_set_damping_scheme.argtypes = [C.c_void_p, C.c_int]
        L.tlsph_set_divergence.argtypes = [C.c_void_p, C.c_double]
        L.tlsph_get_von_mises.argtypes = [C.c_void_p, _dp]
        L.tlsph_get_von_mises_noalloc.argtypes = [C.c_void_p, _dp]
        L.tlsph_relax_until.argtypes = [C.c_void_p, C.c_double, C.c_int64, C.POINTER(_Report)]
        L.tlsph_step.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.POINTER(_Report)]
        L.tlsph_get_displacement.argtypes = [C.c_void_p, _dp]
        L.tlsph_get_state.argtypes = [C.c_void_p, _dp, _dp, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.tlsph_set_state.argtypes = [C.c_void_p, _dp, _dp, C.c_int64, C.c_double]
        L.tlsph_debug_topology.argtypes = [C.c_void_p] + [C.POINTER(C.c_int32)] * 3 + [C.POINTER(C.c_int64),
                                                                                     C.POINTER(C.c_int32)]
        L.tlsph_body_info.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int64)]
        L.tlsph_debug_bricks.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.tlsph_profile.argtypes = [C.c_void_p, C.c_int]
        L.tlsph_profile_read.argtypes = [C.c_void_p, _dp, C.POINTER(C.c_int64), C.c_int]
        L.tlsph_profile_read.restype = C.c_int
        L.tlsph_damping_decisions.argtypes = [C.c_uint64, C.c_double, C.c_int64, C.c_int64, C.POINTER(C.c_uint8)]
        L.tlsph_destroy_body.argtypes = [C.c_void_p]
        L.tlsph_destroy_body.restype = None
        L.tlsph_server_create.argtypes = [C.c_size_t, C.c_int, C.c_int, C.c_void_p, _Allocator, C.POINTER(C.c_void_p)]
        L.tlsph_server_submit.argtypes = [C.c_void_p, C.POINTER(_Request), C.POINTER(C.c_int64)]
        L.tlsph_server_wait.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                        C.POINTER(_Report)]
        L.tlsph_server_result.argtypes = [C.c_void_p, C.c_int64, _dp]
        L.tlsph_server_times.argtypes = [C.c_void_p, C.c_int64, _dp]
        L.tlsph_server_error.argtypes = [C.c_void_p, C.c_int64]
        L.tlsph_server_error.restype = C.c_char_p
        L.tlsph_server_stats_get.argtypes = [C.c_void_p, C.POINTER(_ServerStats)]
        L.tlsph_server_destroy.argtypes = [C.c_void_p]
        L.tlsph_server_destroy.restype = None
        _lib = L
    return _lib


def last_error() -> str:
    return lib().tlsph_last_error().decode()


def version() -> str:
    return lib().tlsph_version().decode()


def _check(code: int, ok=(OK,)) -> int:
    if code not in ok:
        raise TLSPHError(code, last_error())
    return code


def _ptr(a: Optional[np.ndarray], ty=_dp):
    return None if a is None else a.ctypes.data_as(ty)


def damping_decisions(seed: int, alpha: float, n0: int, count: int) -> np.ndarray:
    """Random-choice decisions (1 = damped) of steps n0 .. n0 + count - 1 (host only)."""
    out = np.zeros(count, np.uint8)
    _check(lib().tlsph_damping_decisions(seed, alpha, n0, count, _ptr(out, C.POINTER(C.c_uint8))))
    return out


# ------------------------------------------------------------------------------------------------
# torch-backed device memory and streams
# ------------------------------------------------------------------------------------------------
class _TorchAllocator:
    """Device memory from torch's caching allocator, on the body's device and stream."""

    def __init__(self, device, stream):
        self.device = device
        self.stream = stream
        self.c_alloc = _ALLOC_FN(self._alloc)
        self.c_free = _FREE_FN(self._free)
        self.struct = _Allocator(self.c_alloc, self.c_free, None)

    def _alloc(self, nbytes, ctx):
        import torch
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), device=self.device, stream=self.stream))
        except Exception:  # out of memory -> NULL; the library reports TLSPH_E_NOMEM
            return None

    def _free(self, ptr, ctx):
        import torch
        if ptr:
            torch.cuda.caching_allocator_delete(int(ptr))


def _report(r: _Report, status: int) -> dict:
    return dict(status=status, steps=r.steps, damped_steps=r.damped_steps, step_index=r.step_index,
                residual=r.residual, kinetic_energy=r.kinetic_energy, force_residual=r.force_residual, dt=r.dt,
                wall_s=r.wall_s, window=r.window, converged=bool(r.converged))


class Body:
    """A relaxation body on one GPU (``tlsph_create_body`` and the calls that take its handle)."""

    def __init__(self, dim: int, X0: np.ndarray, clamped: Optional[np.ndarray], dp: float, h_over_dp: float = 1.3,
                 rho0: float = 1000.0, precision: int = FP32, device=None, stream=None, use_torch=True):
        X0 = np.ascontiguousarray(X0, dtype=np.float64)
        self.dim, self.n = int(dim), int(X0.shape[0])
        self.precision = int(precision)
        cl = None if clamped is None else np.ascontiguousarray(clamped, dtype=np.uint8)
        self._alloc = None
        stream_ptr = None
        alloc = _Allocator(_ALLOC_FN(), _FREE_FN(), None)
        if use_torch:
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("no GPU visible to torch (the library has no CPU path)")
            device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
            stream = torch.cuda.current_stream(device) if stream is None else stream
            self.torch_stream = stream
            stream_ptr = stream.cuda_stream
            self._alloc = _TorchAllocator(device.index, stream)
            alloc = self._alloc.struct
        desc = _BodyDesc(self.dim, self.n, _ptr(X0), _ptr(cl, C.POINTER(C.c_uint8)), dp, h_over_dp, rho0,
                         self.precision, stream_ptr, alloc)
        h = C.c_void_p()
        _check(lib().tlsph_create_body(C.byref(desc), C.byref(h)))
        self._h = h
        self.clamped = np.zeros(self.n, np.uint8) if cl is None else cl.copy()

    # -- lifecycle
    def destroy_body(self):
        if getattr(self, "_h", None):
            lib().tlsph_destroy_body(self._h)
            self._h = None

    close = destroy_body

    def __del__(self):
        try:
            self.destroy_body()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.destroy_body()

    # -- parameters
    def set_material(self, model, E: float, nu: float):
        m = MODELS[model] if isinstance(model, str) else int(model)
        _check(lib().tlsph_set_material(self._h, m, E, nu))

    def set_loads(self, g, accel: Optional[np.ndarray] = None):
        g = np.ascontiguousarray(np.asarray(g, dtype=np.float64)[: self.dim])
        a = None if accel is None else np.ascontiguousarray(accel, dtype=np.float64).reshape(self.n, self.dim)
        _check(lib().tlsph_set_loads(self._h, _ptr(g), _ptr(a)))

    def set_damping(self, eta: float, beta: float, Lc: float, alpha: float, seed: int):
        _check(lib().tlsph_set_damping(self._h, eta, beta, Lc, alpha, seed))

    def set_damping_scheme(self, scheme):
        """"pairwise" (Sec. 3.2, default) or "particle" (Sec. 3.1, with the time-step limit of Eq. 35)."""
        _check(lib().tlsph_set_damping_scheme(self._h, SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)))

    def set_divergence(self, factor: float):
        """A step whose kinetic energy exceeds factor x the peak it first turned over from fails
        with E_DIVERGED (default factor 1e6)."""
        _check(lib().tlsph_set_divergence(self._h, factor))

    # -- stepping
    def relax_until(self, tol: float, max_steps: int) -> dict:
        r = _Report()
        st = _check(lib().tlsph_relax_until(self._h, tol, max_steps, C.byref(r)), ok=(OK, NOT_CONVERGED))
        return _report(r, st)

    def step(self, nsteps: int = 1, force_damping: int = -1) -> dict:
        r = _Report()
        st = _check(lib().tlsph_step(self._h, nsteps, force_damping, C.byref(r)))
        return _report(r, st)

    # -- state
    def get_displacement(self) -> np.ndarray:
        u = np.zeros((self.n, self.dim))
        _check(lib().tlsph_get_displacement(self._h, _ptr(u)))
        return u

    def get_von_mises(self) -> np.ndarray:
        """Von Mises stress of every particle for the current displacement (input order)."""
        vm = np.zeros(self.n)
        _check(lib().tlsph_get_von_mises(self._h, _ptr(vm)))
        return vm

    def get_von_mises_noalloc(self) -> np.ndarray:
        """The same field through the entry point that allocates no device memory (bodies of at most
        2^21 particles)."""
        vm = np.zeros(self.n)
        _check(lib().tlsph_get_von_mises_noalloc(self._h, _ptr(vm)))
        return vm

    def get_state(self):
        u = np.zeros((self.n, self.dim))
        v = np.zeros((self.n, self.dim))
        step = C.c_int64()
        dt = C.c_double()
        _check(lib().tlsph_get_state(self._h, _ptr(u), _ptr(v), C.byref(step), C.byref(dt)))
        return u, v, step.value, dt.value

    def set_state(self, u=None, v=None, step: int = 0, dt: float = 0.0):
        u = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(self.n, self.dim)
        v = None if v is None else np.ascontiguousarray(v, dtype=np.float64).reshape(self.n, self.dim)
        _check(lib().tlsph_set_state(self._h, _ptr(u), _ptr(v), step, dt))

    def debug_topology(self) -> dict:
        n, nnz, _, _ = self.body_info()
        perm = np.zeros(n, np.int32)
        cell = np.zeros(n, np.int32)
        colour = np.zeros(n, np.int32)
        row_ptr = np.zeros(n + 1, np.int64)
        col = np.zeros(max(nnz, 1), np.int32)
        i32 = C.POINTER(C.c_int32)
        _check(lib().tlsph_debug_topology(self._h, _ptr(perm, i32), _ptr(cell, i32), _ptr(colour, i32),
                                          _ptr(row_ptr, C.POINTER(C.c_int64)), _ptr(col, i32)))
        return dict(perm=perm, cell=cell, colour=colour, row_ptr=row_ptr, col=col[:nnz])

    def body_info(self):
        n, nnz, win = C.c_int64(), C.c_int64(), C.c_int64()
        nc = (C.c_int32 * 3)()
        _check(lib().tlsph_body_info(self._h, C.byref(n), C.byref(nnz), nc, C.byref(win)))
        return n.value, nnz.value, tuple(nc), win.value

    @property
    def nnz(self) -> int:
        return self.body_info()[1]

    def debug_bricks(self):
        """(cells per brick of the F / stress pass, cells per brick of the pair-force pass)."""
        a, b = C.c_int32(), C.c_int32()
        _check(lib().tlsph_debug_bricks(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    # -- profiling
    def profile(self, enable: bool = True):
        _check(lib().tlsph_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        ms = np.zeros(8)
        cnt = np.zeros(8, np.int64)
        k = lib().tlsph_profile_read(self._h, _ptr(ms), _ptr(cnt, C.POINTER(C.c_int64)), 8)
        return {PASS_NAMES[i]: (float(ms[i]), int(cnt[i])) for i in range(k)}


def create_body(dim, X0, clamped, dp, h_over_dp=1.3, rho0=1000.0, precision=FP32, **kw) -> Body:
    return Body(dim, X0, clamped, dp, h_over_dp, rho0, precision, **kw)


def from_workload(wb, precision: int = FP32, **kw) -> Body:
    """Creates and configures a body from a ``workloads.Body`` description."""
    b = Body(wb.dim, wb.X0, wb.clamped, wb.dp, wb.h_over_dp, wb.rho0, precision, **kw)
    b.set_material(wb.model, wb.E, wb.nu)
    b.set_loads(wb.g3()[: wb.dim], wb.accel)
    b.set_damping(-1.0, wb.beta, wb.Lc, wb.alpha, wb.seed)
    b.set_damping_scheme(getattr(wb, "scheme", "pairwise"))
    return b


class Server:
    """Continuous-batching request server (``tlsph_server_*``): requests are admitted by memory
    budget into one batched relaxation loop on the GPU.  The pool of ``hbm_budget`` bytes comes from
    torch's caching allocator; the 3D bodies run on torch's current stream."""

    def __init__(self, hbm_budget: int, max_slots: int = 32, precision: int = FP32, device=None):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        stream = torch.cuda.current_stream(dev)
        self._alloc = _TorchAllocator(dev, stream)
        self.precision = int(precision)
        self._inputs = {}
        h = C.c_void_p()
        _check(lib().tlsph_server_create(int(hbm_budget), int(max_slots), self.precision,
                                         C.c_void_p(stream.cuda_stream), self._alloc.struct, C.byref(h)))
        self._h = h

    def submit(self, wb, tol: Optional[float] = None, max_steps: Optional[int] = None) -> int:
        """Queues the relaxation of a ``workloads.Body``; returns its ticket."""
        X0 = np.ascontiguousarray(wb.X0, dtype=np.float64)
        cl = None if wb.clamped is None else np.ascontiguousarray(wb.clamped, dtype=np.uint8)
        acc = None if wb.accel is None else np.ascontiguousarray(wb.accel, dtype=np.float64)
        q = _Request()
        q.body.dim = wb.dim
        q.body.n = X0.shape[0]
        q.body.X0 = _ptr(X0)
        q.body.clamped = _ptr(cl, C.POINTER(C.c_uint8))
        q.body.dp = wb.dp
        q.body.h_over_dp = wb.h_over_dp
        q.body.rho0 = wb.rho0
        q.model = MODELS[wb.model] if isinstance(wb.model, str) else int(wb.model)
        q.E, q.nu = wb.E, wb.nu
        g = wb.g3()
        for k in range(3):
            q.g[k] = float(g[k]) if k < wb.dim else 0.0
        q.accel = _ptr(acc)
        q.eta, q.beta, q.Lc, q.alpha, q.seed = -1.0, wb.beta, wb.Lc, wb.alpha, wb.seed
        q.tol = wb.tol if tol is None else tol
        q.max_steps = wb.max_steps if max_steps is None else max_steps
        q.scheme = SCHEMES[getattr(wb, "scheme", "pairwise")]
        t = C.c_int64()
        _check(lib().tlsph_server_submit(self._h, C.byref(q), C.byref(t)))
        self._inputs[t.value] = (X0.shape[0], wb.dim)
        return t.value

    def wait(self, ticket: int, timeout: float = 0.0):
        """None while running, else the report dict (status OK / NOT_CONVERGED / error code)."""
        done, st, r = C.c_int(), C.c_int(), _Report()
        _check(lib().tlsph_server_wait(self._h, ticket, float(timeout), C.byref(done), C.byref(st), C.byref(r)))
        if not done.value:
            return None
        rep = _report(r, st.value)
        if st.value < 0:
            rep["error"] = lib().tlsph_server_error(self._h, ticket).decode()
        return rep

    def result(self, ticket: int) -> np.ndarray:
        n, dim = self._inputs[ticket]
        u = np.empty((n, dim), np.float64)
        _check(lib().tlsph_server_result(self._h, ticket, _ptr(u)))
        return u

    def times(self, ticket: int) -> np.ndarray:
        """[submitted, setup started, joined the batch, result ready], seconds since creation."""
        t = np.empty(4, np.float64)
        _check(lib().tlsph_server_times(self._h, ticket, _ptr(t)))
        return t

    def stats(self) -> dict:
        s = _ServerStats()
        _check(lib().tlsph_server_stats_get(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in _ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().tlsph_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
