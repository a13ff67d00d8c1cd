"""Parity on the benchmark's headline body: the 3D column of 200 x 200 x 1000 free particles plus 4
clamped base layers (40,160,000 particles, 3,178,450,616 CSR entries), in the launch configuration
bench.py times.  This is where code paths run that smaller bodies never reach: CSR offsets past
2^31 (row offsets are 64-bit, every slot and damping factor is indexed through them) and the 4-cell
bricks of both pair passes that bodies above 8M particles take.  The oracle (in its
shared-memory mode, bit-identical to the serial oracle) builds the same body: the neighbour lists,
cells and colours must match bit for bit, and one step (plain, then damped) from a smooth state must
match element-wise within the FP32 bar, and within 1e-10 in FP64."""
import math
import os
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


def _threads():
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return max(1, min(16, usable))


@pytest.fixture(scope="module")
def body():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return workloads.c5_column()


@pytest.fixture(scope="module")
def oracle_body(body):
    oracle.set_threads(_threads())
    _say(f"oracle setup of the 40.16M-particle column ({oracle.threads()} threads)")
    ob = oracle.OracleBody(body)
    yield ob
    ob.close()
    oracle.set_threads(1)


def smooth_state(body, seed=0):
    """Bending-like smooth displacement along the column (quadratic in z) and a smooth velocity."""
    rng = np.random.default_rng(seed)
    X = body.X0 - body.X0.min(axis=0)
    L = X.max(axis=0) + body.dp
    z = X[:, 2] / L[2]
    u = np.zeros_like(X)
    u[:, 0] = 0.02 * z * z + 1e-4 * np.sin(2 * math.pi * X[:, 1] / L[1])
    u[:, 2] = 1e-3 * z * (X[:, 0] / L[0] - 0.5)
    v = 0.01 * np.sin(math.pi * X / L) @ rng.standard_normal((3, 3)).T
    u[body.clamped == 1] = 0
    v[body.clamped == 1] = 0
    return u, v


def test_column_topology_bit_exact(body, oracle_body):
    _say("column topology")
    with tl.from_workload(body, precision=32) as gb:
        n, nnz, _, _ = gb.body_info()
        assert gb.debug_bricks() == (4, 4)          # the 4-cell bricks of bodies above 8M particles
        got = gb.debug_topology()
    assert n == 40_160_000 and nnz == 3_178_450_616 and nnz > 2**31
    ref = oracle_body.topology()
    for k in ("perm", "cell", "colour", "row_ptr"):
        assert np.array_equal(got[k].astype(np.int64), ref[k]), k
    del got["perm"], got["cell"], got["colour"]
    gc, rc = got["col"], ref["col"]
    assert gc.shape == rc.shape
    step = 1 << 27
    for a in range(0, gc.shape[0], step):           # in pieces: the arrays hold 3.2e9 entries
        assert np.array_equal(gc[a:a + step].astype(np.int64), rc[a:a + step]), a


@pytest.fixture(scope="module")
def oracle_step(body, oracle_body):
    """One oracle step from the smooth state, plain (force 0) or damped (force 1), computed once."""
    cache = {}

    def get(force):
        if force not in cache:
            _say(f"oracle column step force={force}")
            u0, v0 = smooth_state(body)
            oracle_body.set_state(u0, v0, step=5, dt=1e-5)
            oracle_body.step(1, force=force)
            uo, vo = oracle_body.get_state()
            cache[force] = (u0, v0, uo, vo, oracle_body.dt)
        return cache[force]
    return get


# FP32 (the benchmark's precision) and plain FP64, whose pass B also takes compact neighbourhoods here
@pytest.mark.parametrize("precision,tol", [(32, 1e-4), (64, 1e-10)], ids=["fp32", "fp64"])
@pytest.mark.parametrize("force", [0, 1])
def test_column_one_step(body, oracle_step, force, precision, tol):
    _say(f"column one FP{precision} step force={force}")
    u0, v0, uo, vo, dto = oracle_step(force)
    with tl.from_workload(body, precision=precision) as gb:
        gb.set_state(u0, v0, step=5, dt=1e-5)
        rep = gb.step(1, force_damping=force)
        ug, vg, step, dt = gb.get_state()
    assert step == 6 and rep["damped_steps"] == force
    ev, eu = rel(vg - v0, vo - v0), rel(ug - u0, uo - u0)
    _say(f"  rel err dv {ev:.3e} du {eu:.3e}")
    assert ev < tol and eu < tol
    assert dt == pytest.approx(dto, rel=max(tol, 1e-12))
