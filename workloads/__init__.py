"""Seeded synthetic bodies for the splitting random-choice dynamic relaxation.

This module only builds inputs: lattice positions, clamp flags, loads and the
material/damping parameters of each workload.  It holds none of the method's
arithmetic, so both the FP64 oracle (``oracle/``) and the HIP library
(``paper_2103_08932_amd``) can be fed from it without sharing any code.

The paper's own bodies (Sec. 4) exist only in missing figures, so every
workload is a regular lattice stand-in: particle ``(i, j[, k])`` sits at
``((i + 1/2) dp, (j + 1/2) dp[, (k + 1/2) dp])`` and clamped layers are extra
lattice layers at negative indices on the clamped face.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

MODELS = ("svk", "nh")


@dataclasses.dataclass
class Body:
    """One relaxation problem: reference configuration, material, loads, damping."""

    name: str
    dim: int
    X0: np.ndarray            # (n, dim) float64, input order
    clamped: np.ndarray       # (n,) uint8, 1 = clamped (Dirichlet u = v = 0)
    dp: float
    h_over_dp: float = 1.3    # Sec. 4: h = 1.3 dp
    rho0: float = 1000.0
    model: str = "nh"         # "svk" (Eq. 4) or "nh" (Eqs. 7-8)
    E: float = 1e6
    nu: float = 0.3
    g: Sequence[float] = (0.0, 0.0, 0.0)
    accel: Optional[np.ndarray] = None   # (n, dim) float64 extra per-particle load, or None
    beta: float = 1.0          # Eq. 36 shape parameter
    Lc: float = 0.0            # Eq. 36 characteristic length
    alpha: float = 0.2         # Eq. 40 random-choice probability
    seed: int = 0              # random-choice stream key
    scheme: str = "pairwise"   # damping scheme: "pairwise" (Sec. 3.2) or "particle" (Sec. 3.1)
    tol: float = 1e-4
    max_steps: int = 10_000
    lattice_shape: tuple = ()  # free-lattice extent, for bookkeeping

    @property
    def n(self) -> int:
        return int(self.X0.shape[0])

    @property
    def n_free(self) -> int:
        return int(self.n - int(self.clamped.sum()))

    def g3(self) -> np.ndarray:
        g = np.zeros(3)
        g[: len(self.g)] = self.g
        return g


def lattice_points(shape: Sequence[int], lo: Sequence[int], dp: float) -> np.ndarray:
    """Cell-centred lattice points for index ranges lo[a] <= idx < lo[a] + shape[a]."""
    axes = [(np.arange(lo[a], lo[a] + shape[a], dtype=np.float64) + 0.5) * dp for a in range(len(shape))]
    grids = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.reshape(-1) for g in grids], axis=1)


def lattice_indices(shape: Sequence[int], lo: Sequence[int]) -> np.ndarray:
    axes = [np.arange(lo[a], lo[a] + shape[a], dtype=np.int64) for a in range(len(shape))]
    grids = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.reshape(-1) for g in grids], axis=1)


def cantilever(dim: int, nfree: Sequence[int], dp: float, nclamp: int = 4, clamp_axis: int = 0,
               jitter: float = 0.0, jitter_seed: int = 0, name: str = "cantilever", **kw) -> Body:
    """Block of ``nfree`` lattice particles with ``nclamp`` clamped layers below index 0
    along ``clamp_axis``.  ``jitter`` is the half-width of a uniform per-component
    perturbation, in units of dp, applied to every particle."""
    nfree = tuple(int(x) for x in nfree)
    assert len(nfree) == dim
    free_idx = lattice_indices(nfree, (0,) * dim)
    cshape = list(nfree)
    cshape[clamp_axis] = nclamp
    clo = [0] * dim
    clo[clamp_axis] = -nclamp
    clamp_idx = lattice_indices(cshape, clo) if nclamp > 0 else np.zeros((0, dim), np.int64)
    idx = np.concatenate([free_idx, clamp_idx], axis=0)
    X0 = (idx.astype(np.float64) + 0.5) * dp
    if jitter > 0.0:
        X0 = X0 + dp * _lattice_jitter(idx, jitter, jitter_seed, lo=tuple(min(0, c) for c in clo),
                                         shape=tuple(nfree[a] + (nclamp if a == clamp_axis else 0)
                                                     for a in range(dim)))
    clamped = np.concatenate([np.zeros(len(free_idx), np.uint8), np.ones(len(clamp_idx), np.uint8)])
    return Body(name=name, dim=dim, X0=np.ascontiguousarray(X0), clamped=clamped, dp=dp,
                lattice_shape=nfree, **kw)


def _lattice_jitter(idx: np.ndarray, half_width: float, seed: int, lo, shape) -> np.ndarray:
    """Uniform(-half_width, half_width) per component, drawn for the whole index box
    ``lo .. lo + shape`` from numpy's Philox generator (key = seed), so any crop of
    the same box sees the same values."""
    dim = idx.shape[1]
    rng = np.random.Generator(np.random.Philox(key=seed))
    full = rng.uniform(-half_width, half_width, size=tuple(shape) + (dim,))
    rel = idx - np.asarray(lo, dtype=np.int64)[None, :]
    return full[tuple(rel[:, a] for a in range(dim))]


# ---------------------------------------------------------------------------------------------
# Named workloads.  Material / load / damping parameters follow the workload definitions; the
# artificial viscosity is given as (beta, Lc) for Eq. 36 with Lc = the body's thickness.
# ---------------------------------------------------------------------------------------------

def c1_cantilever_2d(model: str = "svk", g: float = 9.81, **over) -> Body:
    """2D clamped cantilever, 0.2 x 0.02 m, dp = 0.002: 100 x 10 free + 4 x 10 clamped."""
    kw = dict(name="cantilever2d_1040", model=model, E=1e6, nu=0.3, rho0=1000.0, g=(0.0, -g),
              beta=1.0, Lc=0.02, alpha=0.2, seed=0, tol=1e-6, max_steps=10_000)
    kw.update(over)
    return cantilever(2, (100, 10), 0.002, nclamp=4, **kw)


def c2_cantilever_3d(nx: int = 500, ny: int = 50, nz: int = 50, dp: float = 0.002, **over) -> Body:
    """3D clamped cantilever 1.0 x 0.1 x 0.1 m, dp = 0.002: 500 x 50 x 50 free + 4 clamped layers
    (other nx, ny, nz, dp give other sizes or resolutions)."""
    kw = dict(name=f"cantilever3d_{nx}x{ny}x{nz}", model="nh", E=1e6, nu=0.3, rho0=1000.0,
              g=(0.0, -9.81, 0.0), beta=1.0, Lc=min(ny, nz) * dp, alpha=0.2, seed=1, tol=1e-4,
              max_steps=400_000)
    kw.update(over)
    return cantilever(3, (nx, ny, nz), dp, nclamp=4, **kw)


def c3_block(n: int = 160, crop: Optional[int] = None, **over) -> Body:
    """3D compressed block, 0.4^3 m at dp = 0.0025 (160^3), lattice jittered by U(-0.1, 0.1) dp.
    Bottom (y < 0) clamped by 4 layers; the top free layer carries a downward traction of 1e4 Pa
    applied as the per-particle acceleration t / (rho0 dp).  ``crop`` keeps lattice indices
    [0, crop)^3 of the same jittered lattice (same jitter values) plus its own clamped layers."""
    dp = 0.0025
    rho0 = 1000.0
    m = n if crop is None else int(crop)
    nclamp = 4
    # Jitter is drawn over the full (n, n + 4, n) box so crops reuse the identical values.
    free_idx = lattice_indices((m, m, m), (0, 0, 0))
    clamp_idx = lattice_indices((m, nclamp, m), (0, -nclamp, 0))
    idx = np.concatenate([free_idx, clamp_idx], axis=0)
    jit = _lattice_jitter(idx, 0.1, 0, lo=(0, -nclamp, 0), shape=(n, n + nclamp, n))
    X0 = (idx.astype(np.float64) + 0.5) * dp + dp * jit
    clamped = np.concatenate([np.zeros(len(free_idx), np.uint8), np.ones(len(clamp_idx), np.uint8)])
    accel = np.zeros((len(idx), 3))
    top = idx[:, 1] == m - 1
    accel[top, 1] = -1e4 / (rho0 * dp)
    kw = dict(name=f"block3d_{m}cubed" + ("" if crop is None else f"_crop_of_{n}"), model="nh", E=1e6,
              nu=0.45, rho0=rho0, g=(0.0, 0.0, 0.0), beta=1.0, Lc=m * dp, alpha=0.2, seed=0, tol=1e-4,
              max_steps=200_000)
    kw.update(over)
    return Body(dim=3, X0=np.ascontiguousarray(X0), clamped=clamped, dp=dp, accel=accel,
                lattice_shape=(m, m, m), **kw)


def c5_column(nx: int = 200, ny: int = 200, nz: int = 1000, **over) -> Body:
    """Large 3D clamped column 0.2 x 0.2 x 1.0 m, dp = 0.001, base (z < 0) clamped, lateral +x load."""
    dp = 0.001
    kw = dict(name=f"column3d_{nx}x{ny}x{nz}", model="nh", E=5e6, nu=0.3, rho0=1000.0,
              g=(5.0, 0.0, 0.0), beta=1.0, Lc=min(nx, ny) * dp, alpha=0.2, seed=3, tol=1e-4,
              max_steps=400_000)
    kw.update(over)
    return cantilever(3, (nx, ny, nz), dp, nclamp=4, clamp_axis=2, **kw)


def twisting_cantilever_3d(nx: int = 30, ny: int = 12, nz: int = 12, d: float = 0.04, **over) -> Body:
    """The twisting cantilever of Sec. 4.2: the bending example's neo-Hookean beam (rho0 = 1265,
    E = 5e4 Pa, nu = 0.45; cross-section d x d with d = 0.04 m, length 2.5 d, the d / l = 0.4 of
    its beta; 12 particles through the thickness) clamped at its x = 0 end by 4 layers, under the
    rotational body force of Eq. 41 read as the rotation about the beam axis
    b = (0, -z' gamma, y' gamma) with gamma = (20 g / d) sin(pi x / (2 L)), g = 9.8 m/s^2, L the free
    length and (y', z') the offsets from the cross-section's centre line, taken in the reference
    configuration (a dead load).  No gravity."""
    dp = d / ny
    kw = dict(name=f"twisting3d_{nx}x{ny}x{nz}", model="nh", E=5e4, nu=0.45, rho0=1265.0,
              g=(0.0, 0.0, 0.0), beta=1.0, Lc=d, alpha=0.2, seed=5, tol=1e-4, max_steps=200_000)
    kw.update(over)
    body = cantilever(3, (nx, ny, nz), dp, nclamp=4, **kw)
    X = body.X0
    L = nx * dp
    yc, zc = 0.5 * ny * dp, 0.5 * nz * dp
    gam = 20.0 * 9.8 / d * np.sin(np.pi * X[:, 0] / (2.0 * L))
    acc = np.zeros_like(X)
    acc[:, 1] = -(X[:, 2] - zc) * gam
    acc[:, 2] = (X[:, 1] - yc) * gam
    acc[body.clamped == 1] = 0.0
    body.accel = acc
    return body


def small_body(dim: int, shape: Sequence[int], dp: float = 0.002, nclamp: int = 2, jitter: float = 0.0,
               jitter_seed: int = 0, **over) -> Body:
    """Small cantilever-like body for parity and pin tests."""
    kw = dict(name=f"small{dim}d_" + "x".join(str(s) for s in shape), model="nh", E=1e6, nu=0.3,
              rho0=1000.0, g=(0.0, -9.81) if dim == 2 else (0.0, -9.81, 0.0), beta=1.0,
              Lc=min(shape[1:]) * dp if dim > 1 else shape[0] * dp, alpha=0.2, seed=7, tol=1e-4,
              max_steps=1000)
    kw.update(over)
    return cantilever(dim, shape, dp, nclamp=nclamp, jitter=jitter, jitter_seed=jitter_seed, **kw)


# ---------------------------------------------------------------------------------------------
# Serving stream: Poisson arrivals of relaxation requests of uneven size.
# ---------------------------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after stream start
    body: Body


def _request_uniforms(seed: int, rid: int, count: int = 8) -> np.ndarray:
    """``count`` uniforms in [0, 1) for request ``rid``: numpy's Philox keyed by the stream seed,
    counter (rid, 0, 0, 2), independent of every other request."""
    bg = np.random.Philox(key=seed, counter=[rid, 0, 0, 2])
    raw = bg.random_raw(count)
    return (raw >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def serving_request(rid: int, seed: int = 2, n_lo: float = 5e3, n_hi: float = 5e5) -> Body:
    """One request of the serving stream: 2D or 3D (p = 1/2), log-uniform particle count, 10:1
    cantilever (2D), 10:1:1 cantilever or 10:10:1 plate (3D), log-uniform E in [1e5, 1e7] Pa,
    uniform nu in [0.25, 0.45], uniform gravity magnitude in [1, 20] m/s^2 along -y."""
    u = _request_uniforms(seed, rid)
    dim = 2 if u[0] < 0.5 else 3
    n_target = math.exp(math.log(n_lo) + u[1] * (math.log(n_hi) - math.log(n_lo)))
    E = math.exp(math.log(1e5) + u[2] * (math.log(1e7) - math.log(1e5)))
    nu = 0.25 + 0.2 * u[3]
    gmag = 1.0 + 19.0 * u[4]
    dp = 0.002
    if dim == 2:
        nx = max(10, int(round(math.sqrt(10.0 * n_target))))
        shape = (nx, max(2, nx // 10))
        g = (0.0, -gmag)
    else:
        plate = u[5] >= 0.5
        if plate:  # 10 x 10 x 1 plate, thickness along y
            t = max(2, int(round((n_target / 100.0) ** (1.0 / 3.0))))
            shape = (10 * t, t, 10 * t)
        else:      # 10 x 1 x 1 cantilever
            t = max(2, int(round((n_target / 10.0) ** (1.0 / 3.0))))
            shape = (10 * t, t, t)
        g = (0.0, -gmag, 0.0)
    Lc = min(shape[1:]) * dp
    return cantilever(dim, shape, dp, nclamp=4, name=f"request{rid}", model="nh", E=E, nu=nu,
                      rho0=1000.0, g=g, beta=1.0, Lc=Lc, alpha=0.2, seed=rid, tol=1e-4,
                      max_steps=2_000_000)


def arrival_times(n_requests: int, rate_hz: float, seed: int = 2) -> np.ndarray:
    """Poisson arrival times (seconds, first at 0) at ``rate_hz``: exponential gaps from numpy's
    Philox, key = seed, counter stream 3."""
    bg = np.random.Philox(key=seed, counter=[0, 0, 0, 3])
    gaps = np.random.Generator(bg).exponential(1.0 / rate_hz, size=n_requests)
    return np.cumsum(gaps) - gaps[0]


def serving_stream(n_requests: int, rate_hz: float, seed: int = 2, **kw) -> list:
    """The first ``n_requests`` requests with their Poisson arrival times at ``rate_hz``."""
    t = arrival_times(n_requests, rate_hz, seed)
    return [Request(r, float(t[r]), serving_request(r, seed=seed, **kw)) for r in range(n_requests)]
