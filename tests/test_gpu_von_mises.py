"""GPU parity of the von Mises stress output (the field of the twisting example, Sec. 4.2) against
the FP64 oracle, and of the twisting cantilever workload (Eq. 41 body force) itself."""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads
from parity_metrics import rel

pytestmark = pytest.mark.gpu
tl = pytest.importorskip("paper_2103_08932_amd")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def smooth_u(body, amp=2e-3, seed=0):
    """A smooth displacement of a few per cent strain: affine + quadratic + one sine mode."""
    rng = np.random.default_rng(seed)
    X = body.X0 - body.X0.min(axis=0)
    L = X.max(axis=0) + body.dp
    D = body.dim
    u = amp * (X @ rng.standard_normal((D, D)).T + (X / L) ** 2 @ rng.standard_normal((D, D)).T * L.max()
               + np.sin(2 * math.pi * X / L) @ rng.standard_normal((D, D)).T * L.max() / 20)
    u[body.clamped == 1] = 0
    return u


def max_rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


CASES = [
    ("2d_svk", dict(dim=2, shape=(30, 8), nclamp=3, jitter=0.1, model="svk")),
    ("2d_nh", dict(dim=2, shape=(30, 8), nclamp=3, jitter=0.1, model="nh")),
    ("3d_nh", dict(dim=3, shape=(14, 6, 7), nclamp=2, jitter=0.15, model="nh")),
    ("3d_svk_lattice", dict(dim=3, shape=(12, 7, 5), nclamp=2, jitter=0.0, model="svk")),
]


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", [64, 32])
def test_von_mises_matches_oracle(name, kw, precision):
    _say(f"von Mises {name} fp{precision}")
    kw = dict(kw)
    dim, shape = kw.pop("dim"), kw.pop("shape")
    body = workloads.small_body(dim, shape, jitter_seed=4, **kw)
    u0 = smooth_u(body, seed=len(name))
    ob = oracle.OracleBody(body)
    ob.set_state(u=u0)
    vo = ob.von_mises()
    with tl.from_workload(body, precision=precision) as gb:
        assert np.array_equal(gb.get_von_mises(), np.zeros(body.n))     # at rest
        gb.set_state(u0, None, step=0)
        vg = gb.get_von_mises()
    e = max_rel(vg, vo)
    _say(f"  max |vm| {np.abs(vo).max():.3e} Pa, max rel err {e:.2e}")
    assert e < (1e-10 if precision == 64 else 1e-4)


def test_von_mises_block_crop():
    """The jittered, nearly incompressible 40^3 block crop (70,400 particles) under a smooth
    compression: FP64 within 1e-10 and FP32 within 1e-4 (relative to the largest value)."""
    body = workloads.c3_block(crop=40)
    X = body.X0 - body.X0.min(axis=0)
    Ly = X[:, 1].max() + body.dp
    u = np.zeros_like(X)
    u[:, 1] = -0.01 * Ly * (X[:, 1] / Ly) ** 2
    u[:, 0] = 2e-3 * X[:, 1] * np.sin(np.pi * X[:, 2] / Ly)
    u[body.clamped == 1] = 0
    ob = oracle.OracleBody(body)
    ob.set_state(u=u)
    vo = ob.von_mises()
    for prec, tol in ((64, 1e-10), (32, 1e-4)):
        with tl.from_workload(body, precision=prec) as gb:
            gb.set_state(u, None, step=0)
            e = max_rel(gb.get_von_mises(), vo)
        _say(f"  block crop fp{prec}: max rel err {e:.2e}")
        assert e < tol


@pytest.mark.parametrize("precision", [64, 32])
def test_inverted_state_is_reported(precision):
    body = workloads.small_body(3, (8, 5, 5), nclamp=0, model="nh")
    with tl.from_workload(body, precision=precision) as gb:
        gb.set_state(-2.5 * body.X0, None, step=0)      # F = -1.5 I: J < 0 everywhere
        with pytest.raises(tl.TLSPHError) as ei:
            gb.get_von_mises()
        assert ei.value.code == tl.E_NONFINITE


def test_twisting_cantilever_trajectory_fp64():
    """300 random-choice steps of the twisting cantilever (Eq. 41 body force, 4,896 particles):
    displacement and von Mises stress within 1e-9 of the oracle, the same damped steps."""
    body = workloads.twisting_cantilever_3d()
    ob = oracle.OracleBody(body)
    nd = ob.step(300)
    uo = ob.get_displacement()
    vo = ob.von_mises()
    with tl.from_workload(body, precision=64) as gb:
        rep = gb.step(300)
        ug = gb.get_displacement()
        vg = gb.get_von_mises()
    eu, ev = rel(ug, uo), max_rel(vg, vo)
    _say(f"twisting: {nd} damped, rel err u {eu:.2e}, vm {ev:.2e}, max vm {vo.max():.3e} Pa")
    assert rep["damped_steps"] == nd
    assert eu < 1e-9 and ev < 1e-9
