"""ctypes binding of the FP64 CPU oracle (``tlsph_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py``.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tlsph_oracle.c")
LIB = os.path.join(HERE, "libtlsph_oracle.so")

OK, NOT_CONVERGED, E_INVALID, E_NOMEM, E_SINGULAR, E_NONFINITE, E_DIVERGED = 0, 1, -1, -2, -3, -5, -6
MODEL = {"svk": 0, "nh": 1}
SCHEMES = {"pairwise": 0, "particle": 1, 0: 0, 1: 1}


# FP64, no FMA contraction, no fast-math; OpenMP for the shared-memory mode (bit-identical to serial)
CFLAGS = ["-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-Wall"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def set_threads(n: int) -> int:
    """Threads of the oracle's shared-memory mode (1 = serial); returns the count in effect."""
    return lib().orc_set_threads(int(n))


def threads() -> int:
    return lib().orc_set_threads(0)


class _Report(C.Structure):
    _fields_ = [("steps", C.c_int64), ("damped_steps", C.c_int64), ("residual", C.c_double),
                ("kinetic_energy", C.c_double), ("force_residual", C.c_double), ("converged", C.c_int)]


_lib = None
_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_u64p = C.POINTER(C.c_uint64)


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = load_library(LIB)
        # serial by default (the plain oracle); set_threads() or TLSPH_ORACLE_THREADS selects the
        # shared-memory mode, whose results are bit-identical
        _lib.orc_set_threads(int(os.environ.get("TLSPH_ORACLE_THREADS", "1")))
    return _lib


def load_library(path: str):
    """Bind the oracle's entry points in the shared library at `path` (the built oracle, or a copy
    compiled from a modified source by a test that plants a mistake in it)."""
    L = C.CDLL(path)
    L.orc_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
    L.orc_damped_decision.argtypes = [C.c_uint64, C.c_int64, C.c_double]
    L.orc_damped_decision.restype = C.c_int
    L.orc_eta.argtypes = [C.c_double] * 4
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_set_threads.restype = C.c_int
    L.orc_eta.restype = C.c_double
    L.orc_wendland.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp]
    L.orc_stress.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, _dp, _dp, _dp]
    L.orc_stress.restype = C.c_int
    L.orc_von_mises.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, _dp, C.POINTER(C.c_double)]
    L.orc_von_mises.restype = C.c_int
    L.orc_body_von_mises.argtypes = [C.c_void_p, _dp]
    L.orc_body_von_mises.restype = C.c_int
    L.orc_pair_op.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, _dp, _dp]
    L.orc_body_create.argtypes = [C.c_int, C.c_int64, _dp, C.c_char_p, C.c_double, C.c_double, C.c_double,
                                  C.POINTER(C.c_int)]
    L.orc_body_create.restype = C.c_void_p
    L.orc_body_destroy.argtypes = [C.c_void_p]
    L.orc_body_set_material.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double]
    L.orc_body_set_loads.argtypes = [C.c_void_p, _dp, _dp]
    L.orc_body_set_damping.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_uint64]
    L.orc_body_set_damping_scheme.argtypes = [C.c_void_p, C.c_int]
    L.orc_body_set_divergence.argtypes = [C.c_void_p, C.c_double]
    L.orc_pbp_local.argtypes = [C.c_int, C.c_double, C.c_int64, _dp, C.c_char_p, _dp, _dp]
    L.orc_pbp_local.restype = None
    L.orc_body_eta.argtypes = [C.c_void_p]
    L.orc_body_eta.restype = C.c_double
    L.orc_body_window.argtypes = [C.c_void_p]
    L.orc_body_window.restype = C.c_int64
    L.orc_body_step.argtypes = [C.c_void_p, C.c_int64, C.c_int, _i64p]
    L.orc_body_relax.argtypes = [C.c_void_p, C.c_double, C.c_int64, C.POINTER(_Report)]
    for name in ("orc_body_n", "orc_body_nnz", "orc_body_step_index"):
        getattr(L, name).argtypes = [C.c_void_p]
        getattr(L, name).restype = C.c_int64
    for name in ("orc_body_dt", "orc_body_residual", "orc_body_kinetic_energy", "orc_body_ek_peak"):
        getattr(L, name).argtypes = [C.c_void_p]
        getattr(L, name).restype = C.c_double
    L.orc_body_grid.argtypes = [C.c_void_p, _i64p, _dp, _dp]
    L.orc_body_get_state.argtypes = [C.c_void_p, _dp, _dp]
    L.orc_body_set_state.argtypes = [C.c_void_p, _dp, _dp, C.c_int64, C.c_double]
    L.orc_body_get_F.argtypes = [C.c_void_p, _dp]
    L.orc_body_get_B0.argtypes = [C.c_void_p, _dp]
    L.orc_body_get_accel.argtypes = [C.c_void_p, _dp, _dp]
    L.orc_body_damp.argtypes = [C.c_void_p, C.c_double, C.c_double]
    L.orc_body_topology.argtypes = [C.c_void_p, _i64p, _i64p, _i64p, _i64p, _i64p]
    L.orc_body_cell_colour.argtypes = [C.c_void_p, C.c_int64]
    L.orc_body_cell_colour.restype = C.c_int64
    return L


def _p(a: Optional[np.ndarray], ty=_dp):
    return None if a is None else a.ctypes.data_as(ty)


def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(_p(c, _u64p), _p(k, _u64p), _p(out, _u64p))
    return out


def damped_decision(seed: int, n: int, alpha: float) -> bool:
    return bool(lib().orc_damped_decision(seed, n, alpha))


def eta(beta: float, rho0: float, E: float, L: float) -> float:
    return lib().orc_eta(beta, rho0, E, L)


def wendland(dim: int, h: float, r: float):
    W, dW = C.c_double(), C.c_double()
    lib().orc_wendland(dim, h, r, C.byref(W), C.byref(dW))
    return W.value, dW.value


def stress(dim: int, model: str, lam: float, mu: float, F: np.ndarray):
    F = np.ascontiguousarray(F, dtype=np.float64).reshape(dim, dim)
    S = np.zeros((dim, dim))
    P = np.zeros((dim, dim))
    st = lib().orc_stress(dim, MODEL[model], lam, mu, _p(F), _p(S), _p(P))
    if st != OK:
        raise ValueError(f"oracle stress failed ({st})")
    return S, P


def von_mises(dim: int, model: str, lam: float, mu: float, F: np.ndarray) -> float:
    """Von Mises stress of the Cauchy stress J^-1 F S F^T (plane strain in 2D)."""
    F = np.ascontiguousarray(F, dtype=np.float64).reshape(dim, dim)
    vm = C.c_double()
    st = lib().orc_von_mises(dim, MODEL[model], lam, mu, _p(F), C.byref(vm))
    if st != OK:
        raise ValueError(f"oracle von Mises failed ({st})")
    return vm.value


def pair_op(dim, mi, mj, B, ci, cj, vi, vj):
    vi = np.array(vi, dtype=np.float64)
    vj = np.array(vj, dtype=np.float64)
    lib().orc_pair_op(dim, mi, mj, B, int(ci), int(cj), _p(vi), _p(vj))
    return vi, vj


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


class OracleBody:
    """An oracle body built from a ``workloads.Body`` (or raw arrays)."""

    def __init__(self, body=None, *, dim=None, X0=None, clamped=None, dp=None, h_over_dp=1.3, rho0=1000.0):
        if body is not None:
            dim, X0, clamped, dp, h_over_dp, rho0 = body.dim, body.X0, body.clamped, body.dp, body.h_over_dp, body.rho0
        self.dim = int(dim)
        X0 = np.ascontiguousarray(X0, dtype=np.float64)
        self.n = X0.shape[0]
        cl = None if clamped is None else np.ascontiguousarray(clamped, dtype=np.uint8)
        st = C.c_int(0)
        L = lib()
        self._h = L.orc_body_create(self.dim, self.n, _p(X0), None if cl is None else cl.ctypes.data_as(C.c_char_p),
                                    dp, h_over_dp, rho0, C.byref(st))
        if not self._h:
            raise OracleError(st.value, "create")
        self.clamped = np.zeros(self.n, np.uint8) if cl is None else cl.copy()
        if body is not None:
            self.configure(body)

    def configure(self, body):
        self.set_material(body.model, body.E, body.nu)
        self.set_loads(body.g3()[: self.dim], body.accel)
        self.set_damping(-1.0, body.beta, body.Lc, body.alpha, body.seed)
        self.set_damping_scheme(getattr(body, "scheme", "pairwise"))

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_body_destroy(self._h)
            self._h = None

    __del__ = close

    def _check(self, st, what):
        if st not in (OK, NOT_CONVERGED):
            raise OracleError(st, what)
        return st

    def set_material(self, model, E, nu):
        self._check(lib().orc_body_set_material(self._h, MODEL[model], E, nu), "set_material")

    def set_loads(self, g, accel=None):
        g = np.ascontiguousarray(np.asarray(g, dtype=np.float64)[: self.dim])
        a = None if accel is None else np.ascontiguousarray(accel, dtype=np.float64).reshape(self.n, self.dim)
        self._check(lib().orc_body_set_loads(self._h, _p(g), _p(a)), "set_loads")

    def set_damping(self, eta, beta, Lc, alpha, seed):
        self._check(lib().orc_body_set_damping(self._h, eta, beta, Lc, alpha, seed), "set_damping")

    def set_damping_scheme(self, scheme):
        """'pairwise' (Sec. 3.2) or 'particle' (particle-by-particle, Sec. 3.1)."""
        self._check(lib().orc_body_set_damping_scheme(self._h, SCHEMES[scheme]), "set_damping_scheme")

    def set_divergence(self, factor):
        """A step whose E_k exceeds factor x the E_peak of the first turn-over fails (E_DIVERGED)."""
        self._check(lib().orc_body_set_divergence(self._h, factor), "set_divergence")

    @property
    def eta(self):
        return lib().orc_body_eta(self._h)

    @property
    def window(self):
        return lib().orc_body_window(self._h)

    @property
    def nnz(self):
        return lib().orc_body_nnz(self._h)

    @property
    def step_index(self):
        return lib().orc_body_step_index(self._h)

    @property
    def dt(self):
        return lib().orc_body_dt(self._h)

    @property
    def residual(self):
        return lib().orc_body_residual(self._h)

    @property
    def kinetic_energy(self):
        return lib().orc_body_kinetic_energy(self._h)

    @property
    def ek_peak(self):
        return lib().orc_body_ek_peak(self._h)

    def grid(self):
        nc = np.zeros(3, np.int64)
        xmin = np.zeros(3)
        rc = C.c_double()
        lib().orc_body_grid(self._h, _p(nc, _i64p), _p(xmin), C.byref(rc))
        return nc, xmin, rc.value

    def step(self, nsteps=1, force=-1):
        nd = C.c_int64(0)
        self._check(lib().orc_body_step(self._h, nsteps, force, C.byref(nd)), "step")
        return nd.value

    def relax(self, tol, max_steps):
        r = _Report()
        st = self._check(lib().orc_body_relax(self._h, tol, max_steps, C.byref(r)), "relax")
        return dict(status=st, steps=r.steps, damped_steps=r.damped_steps, residual=r.residual,
                    kinetic_energy=r.kinetic_energy, force_residual=r.force_residual, converged=bool(r.converged))

    def get_state(self):
        u = np.zeros((self.n, self.dim))
        v = np.zeros((self.n, self.dim))
        lib().orc_body_get_state(self._h, _p(u), _p(v))
        return u, v

    def get_displacement(self):
        return self.get_state()[0]

    def set_state(self, u=None, v=None, step=0, dt=0.0):
        u = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(self.n, self.dim)
        v = None if v is None else np.ascontiguousarray(v, dtype=np.float64).reshape(self.n, self.dim)
        self._check(lib().orc_body_set_state(self._h, _p(u), _p(v), step, dt), "set_state")

    def get_F(self):
        F = np.zeros((self.n, self.dim, self.dim))
        lib().orc_body_get_F(self._h, _p(F))
        return F

    def von_mises(self):
        """Von Mises stress of every particle for the current u (input order)."""
        out = np.zeros(self.n)
        self._check(lib().orc_body_von_mises(self._h, _p(out)), "von_mises")
        return out

    def get_B0(self):
        B = np.zeros((self.n, self.dim, self.dim))
        lib().orc_body_get_B0(self._h, _p(B))
        return B

    def get_accel(self, with_T=False):
        a = np.zeros((self.n, self.dim))
        T = np.zeros((self.n, self.dim, self.dim)) if with_T else None
        self._check(lib().orc_body_get_accel(self._h, _p(a), _p(T)), "get_accel")
        return (a, T) if with_T else a

    def damp(self, eta_t, dt):
        lib().orc_body_damp(self._h, eta_t, dt)

    def topology(self):
        n, nnz = self.n, self.nnz
        perm = np.zeros(n, np.int64)
        cell = np.zeros(n, np.int64)
        colour = np.zeros(n, np.int64)
        row_ptr = np.zeros(n + 1, np.int64)
        col = np.zeros(nnz, np.int64)
        lib().orc_body_topology(self._h, _p(perm, _i64p), _p(cell, _i64p), _p(colour, _i64p), _p(row_ptr, _i64p),
                                _p(col, _i64p))
        return dict(perm=perm, cell=cell, colour=colour, row_ptr=row_ptr, col=col)

    def cell_colour(self, lin):
        return lib().orc_body_cell_colour(self._h, lin)
def pbp_local(dim, m, B, clamped, vi, vj):
    """D_i of the particle-by-particle scheme (Sec. 3.1) on particle i and its neighbours:
    B[q] the coefficients of Eq. 27, clamped[q] the neighbours' flags; returns (vi', vj')."""
    B = np.ascontiguousarray(B, dtype=np.float64)
    cl = np.ascontiguousarray(clamped, dtype=np.uint8)
    vi = np.array(vi, dtype=np.float64, copy=True)
    vj = np.array(vj, dtype=np.float64, copy=True).reshape(len(B), dim)
    lib().orc_pbp_local(dim, m, len(B), _p(B), cl.ctypes.data_as(C.c_char_p), _p(vi), _p(vj))
    return vi, vj


