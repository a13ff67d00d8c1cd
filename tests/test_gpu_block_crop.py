"""Parity on the compressed-block workload's 40^3 crop: the 160^3 block's jittered lattice (jitter
U(-0.1, 0.1) dp, the same values the full block uses) cropped to lattice indices [0, 40)^3 plus its
own 4 clamped layers (70,400 particles), neo-Hookean with nu = 0.45 and a 1e4 Pa traction on the top
layer as a per-particle acceleration.  Jitter makes rows irregular and nearly incompressible material
stiffens the pressure response, so this exercises what the lattice cantilevers do not."""
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
    return workloads.c3_block(crop=40)


@pytest.fixture(scope="module")
def oracle_body(body):
    _say("oracle setup of the 40^3 block crop")
    return oracle.OracleBody(body)




def compressed_state(body, seed=3):
    """A smooth compression of about 1 % with a small shear and a smooth velocity field."""
    rng = np.random.default_rng(seed)
    X = body.X0 - body.X0.min(axis=0)
    L = X.max(axis=0) + body.dp
    y = X[:, 1] / L[1]
    u = np.zeros_like(X)
    u[:, 1] = -0.01 * L[1] * y * y
    u[:, 0] = 2e-3 * L[0] * y * np.sin(np.pi * X[:, 2] / L[2])
    v = 0.01 * np.sin(np.pi * X / L) @ rng.standard_normal((3, 3)).T
    u[body.clamped == 1] = 0
    v[body.clamped == 1] = 0
    return u, v


def test_block_crop_topology_bit_exact(body, oracle_body):
    ref = oracle_body.topology()
    with tl.from_workload(body, precision=32) as gb:
        got = gb.debug_topology()
        n, nnz, _, _ = gb.body_info()
    _say(f"block crop: {n} particles, {nnz} CSR entries")
    assert n == 70400
    for k in ("perm", "cell", "colour", "row_ptr"):
        assert np.array_equal(got[k].astype(np.int64), ref[k]), k
    assert np.array_equal(got["col"], ref["col"].astype(np.int32))


@pytest.mark.parametrize("force", [0, 1])
def test_block_crop_one_step_fp64(body, oracle_body, force):
    u0, v0 = compressed_state(body)
    oracle_body.set_state(u0, v0, step=11, dt=1e-5)
    oracle_body.step(1, force=force)
    uo, vo = oracle_body.get_state()
    with tl.from_workload(body, precision=64) as gb:
        gb.set_state(u0, v0, step=11, dt=1e-5)
        rep = gb.step(1, force_damping=force)
        ug, vg, step, dt = gb.get_state()
    assert step == 12 and rep["damped_steps"] == force
    ev, eu = rel(vg - v0, vo - v0), rel(ug - u0, uo - u0)
    _say(f"  fp64 force={force}: rel err dv {ev:.3e} du {eu:.3e}")
    assert ev < 1e-10 and eu < 1e-10
    assert dt == pytest.approx(oracle_body.dt, rel=1e-12)


def test_block_crop_fp32_tracks_fp64(body):
    """The same random-choice trajectory (300 steps from rest under the traction) in FP32 and FP64
    on the GPU: FP32 stress, force and damping with FP64 displacement stay within 1e-4 relative L2
    early in the transient (the comparison against the oracle itself, after deep relaxation, is the
    next test)."""
    out = {}
    for prec in (64, 32):
        with tl.from_workload(body, precision=prec) as gb:
            rep = gb.step(300)
            out[prec] = (gb.get_displacement(), rep["damped_steps"])
    (u64, d64), (u32, d32) = out[64], out[32]
    e = rel(u32, u64)
    _say(f"  fp32 vs fp64 after 300 steps ({d64} damped): rel L2 {e:.3e}")
    assert d32 == d64
    assert np.linalg.norm(u64) > 0 and e < 1e-4


def test_block_crop_fp32_matches_oracle_over_1500_steps(body):
    """FP32 (stress, force and damping; FP64 displacement and reductions) against the FP64 oracle on
    the nearly incompressible, jittered crop, over the first 1,500 random-choice steps from rest
    (the loading transient and its first decay).  The oracle's state at step 1,500, for the top
    (traction) layer and 4,000 seeded particles, is stored in tests/golden, written by
    make_block_crop_golden.py, which calls only the oracle.  Bars: FP32 1e-4 and FP64 1e-8, relative
    over the sample and element-wise.

    Why not after deep relaxation: this body does not relax.  The particles at the corners and edges
    of the loaded face, which carry the full traction acceleration (4,000 m/s^2) with a fraction of a
    full neighbourhood, are flung out and recaptured every few thousand steps from about step 2,000
    on (kinetic energy up to 0.8 of its first peak, over 99.9 % of it in the top four layers, speeds
    near the sound speed at the top corners), in the oracle as on the GPU, and in FP64 one such event
    eventually inverts a particle (step 19,172 on the GPU).  Past the first burst the trajectories of
    different roundings part ways, so equal-step comparisons there measure the chaos, not the
    arithmetic."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "block_crop_40_1500_steps.npz")
    g = np.load(path, allow_pickle=False)
    assert str(g["workload"]) == body.name
    S, idx, uo = int(g["steps"]), g["idx"], g["u"]
    for prec, tol in ((32, 1e-4), (64, 1e-8)):
        with tl.from_workload(body, precision=prec) as gb:
            rep = gb.step(S)
            u = gb.get_displacement()
        e = rel(u[idx], uo)
        _say(f"  fp{prec} after {S} steps ({rep['damped_steps']} damped; oracle residual {float(g['residual']):.1e}): "
             f"rel err {e:.3e} (max |u| {np.abs(u).max():.3e} m)")
        assert rep["damped_steps"] == int(g["damped"])
        assert e < tol
