"""Parity at the benchmark's full size: the 3D cantilever of 500 x 50 x 50 free particles plus 4
clamped layers (1,260,000 particles, 96,714,816 CSR entries), in the launch configuration bench.py
times.  The oracle finishes its setup and one step of this body in seconds, so every output is
compared, not a sample."""
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


@pytest.fixture(scope="module")
def body():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return workloads.c2_cantilever_3d()


@pytest.fixture(scope="module")
def oracle_body(body):
    _say("oracle setup of the 1.26M-particle cantilever")
    return oracle.OracleBody(body)




def smooth_state(body, seed=0):
    """Bending-like smooth displacement (quadratic in x) and a smooth velocity field."""
    rng = np.random.default_rng(seed)
    X = body.X0 - body.X0.min(axis=0)
    L = X.max(axis=0) + body.dp
    x = X[:, 0] / L[0]
    u = np.zeros_like(X)
    u[:, 1] = -0.05 * x * x + 1e-3 * np.sin(2 * math.pi * X[:, 2] / L[2])
    u[:, 0] = 2e-3 * x * (X[:, 1] / L[1] - 0.5)
    v = 0.02 * np.sin(math.pi * X / L) @ rng.standard_normal((3, 3)).T
    u[body.clamped == 1] = 0
    v[body.clamped == 1] = 0
    return u, v


def test_fullsize_topology_bit_exact(body, oracle_body):
    _say("full-size topology")
    ref = oracle_body.topology()
    with tl.from_workload(body, precision=32) as gb:
        got = gb.debug_topology()
        n, nnz, _, _ = gb.body_info()
    assert nnz == 96714816 and n == 1260000
    for k in ("perm", "cell", "colour", "row_ptr"):
        assert np.array_equal(got[k].astype(np.int64), ref[k]), k
    assert np.array_equal(got["col"], ref["col"].astype(np.int32))


@pytest.fixture(scope="module")
def oracle_step(body, oracle_body):
    """One oracle step from the smooth state, plain (force 0) or damped (force 1), computed once."""
    cache = {}

    def get(force):
        if force not in cache:
            _say(f"oracle step force={force}")
            u0, v0 = smooth_state(body)
            oracle_body.set_state(u0, v0, step=5, dt=5e-5)
            oracle_body.step(1, force=force)
            uo, vo = oracle_body.get_state()
            cache[force] = (u0, v0, uo, vo, oracle_body.dt)
        return cache[force]
    return get


# the launch configuration bench.py times (FP32: 5-cell bricks for F / stress, 3-cell bricks for the
# pair-force sum), FP64, and the 4-cell bricks of both passes (one shared slot array) that bodies
# above 8M particles take
CASES = [(64, 1e-10, "default"), (32, 1e-4, "default"), (32, 1e-4, "long_bricks")]


@pytest.mark.parametrize("precision,tol,variant", CASES, ids=[f"fp{p}-{v}" for p, _, v in CASES])
@pytest.mark.parametrize("force", [0, 1])
def test_fullsize_one_step(body, oracle_step, precision, tol, variant, force, monkeypatch):
    _say(f"full-size one step fp{precision} {variant} force={force}")
    if variant == "long_bricks":
        monkeypatch.setenv("TLSPH_PASSB_LONG_BRICK_N", "1000000")
    u0, v0, uo, vo, dto = oracle_step(force)
    with tl.from_workload(body, precision=precision) as gb:
        cells_a, cells_b = gb.debug_bricks()
        if precision == 32:
            assert (cells_a, cells_b) == ((4, 4) if variant == "long_bricks" else (5, 3))
        gb.set_state(u0, v0, step=5, dt=5e-5)
        rep = gb.step(1, force_damping=force)
        ug, vg, step, dt = gb.get_state()
    assert step == 6 and rep["damped_steps"] == force
    ev, eu = rel(vg - v0, vo - v0), rel(ug - u0, uo - u0)
    _say(f"  rel err dv {ev:.3e} du {eu:.3e}")
    assert ev < tol and eu < tol
    assert dt == pytest.approx(dto, rel=max(tol, 1e-12))


def _threads():
    import os
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return max(1, min(16, usable))


@pytest.fixture(scope="module")
def oracle_trajectory(body):
    """100 random-choice steps of the oracle from rest (the benchmark's start, damping seed and
    alpha), run in its shared-memory mode, which is bit-identical to the serial oracle."""
    oracle.set_threads(_threads())
    _say(f"oracle: 100 steps of the full-size cantilever from rest ({oracle.threads()} threads)")
    ob = oracle.OracleBody(body)
    try:
        for _ in range(10):
            ob.step(10)
            _say(f"  oracle step {ob.step_index}")
        return ob.get_displacement(), ob.step_index
    finally:
        ob.close()
        oracle.set_threads(1)


@pytest.mark.parametrize("precision,tol", [(64, 1e-12), (32, 1e-5)], ids=["fp64", "fp32"])
def test_fullsize_trajectory_100_steps(body, oracle_trajectory, precision, tol):
    """The first 100 steps of the benchmark's own run (from rest, Philox damping decisions, adaptive
    time step): the whole trajectory, not one step from a prescribed state.  FP64 agrees with the
    oracle to rounding (about 2e-15 measured); the FP32 bar allows the step-to-step accumulation
    of single-precision stress and force (about 9e-7 measured)."""
    _say(f"full-size trajectory fp{precision}")
    uo, steps = oracle_trajectory
    with tl.from_workload(body, precision=precision) as gb:
        rep = gb.step(100)
        ug = gb.get_displacement()
    assert steps == 100 and rep["steps"] == 100
    e = rel(ug, uo)
    _say(f"  rel err u {e:.3e}")
    assert e < tol
