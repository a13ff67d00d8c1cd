"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Topology (cell order, colours, CSR rows) must match bit for bit.  Floating point: one step of the
FP64 path from an identical state within 1e-10 relative (over the step's increments of u and v);
the FP32 path within 1e-4 relative on the final displacement after deep relaxation at equal step
counts.  Every relative error is the worse of the field's relative L2 error and its element-wise
max |got - ref| / max |ref| (parity_metrics.rel).
"""
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
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tl.lib()
    yield
    torch.cuda.synchronize()




TOPO_CASES = [
    ("2d_lattice", dict(dim=2, shape=(31, 7), nclamp=3, jitter=0.0)),
    ("2d_jitter", dict(dim=2, shape=(40, 11), nclamp=4, jitter=0.2)),
    ("3d_lattice", dict(dim=3, shape=(19, 6, 7), nclamp=2, jitter=0.0)),
    ("3d_jitter", dict(dim=3, shape=(23, 9, 5), nclamp=4, jitter=0.25)),
    ("3d_ragged", dict(dim=3, shape=(3, 17, 2), nclamp=1, jitter=0.1)),
]


@pytest.mark.parametrize("name,kw", TOPO_CASES, ids=[c[0] for c in TOPO_CASES])
@pytest.mark.parametrize("precision", [32, 64])
def test_topology_bit_exact(name, kw, precision):
    _say(f"topology {name} fp{precision}")
    body = workloads.small_body(kw["dim"], kw["shape"], nclamp=kw["nclamp"], jitter=kw["jitter"], jitter_seed=3)
    ob = oracle.OracleBody(body)
    ref = ob.topology()
    with tl.from_workload(body, precision=precision) as gb:
        got = gb.debug_topology()
    for k in ("perm", "cell", "colour", "row_ptr", "col"):
        assert np.array_equal(got[k].astype(np.int64), ref[k]), k


def smooth_state(body, amp_u=1e-4, amp_v=1e-2, seed=0):
    """A smooth displacement / velocity field: affine + quadratic + one sine mode."""
    rng = np.random.default_rng(seed)
    X = body.X0 - body.X0.min(axis=0)
    L = X.max(axis=0) + body.dp
    D = body.dim
    A = rng.standard_normal((D, D))
    Q = rng.standard_normal((D, D))
    u = amp_u * (X @ A.T / L.max() + (X / L) ** 2 @ Q.T * L.max() / 10)
    v = amp_v * np.sin(2 * math.pi * X / L) @ rng.standard_normal((D, D)).T
    u[body.clamped == 1] = 0
    v[body.clamped == 1] = 0
    return u, v


STEP_CASES = [
    ("2d_svk", dict(dim=2, shape=(30, 8), nclamp=3, jitter=0.1, model="svk")),
    ("2d_nh", dict(dim=2, shape=(30, 8), nclamp=3, jitter=0.1, model="nh")),
    ("3d_nh", dict(dim=3, shape=(14, 6, 7), nclamp=2, jitter=0.15, model="nh")),
    ("3d_svk_lattice", dict(dim=3, shape=(12, 7, 5), nclamp=2, jitter=0.0, model="svk")),
]


@pytest.mark.parametrize("name,kw", STEP_CASES, ids=[c[0] for c in STEP_CASES])
@pytest.mark.parametrize("force", [0, 1])
def test_one_step_fp64(name, kw, force):
    _say(f"one step fp64 {name} force={force}")
    body = workloads.small_body(kw["dim"], kw["shape"], nclamp=kw["nclamp"], jitter=kw["jitter"], jitter_seed=5,
                                model=kw["model"], alpha=0.2)
    u0, v0 = smooth_state(body, seed=len(name))
    ob = oracle.OracleBody(body)
    ob.set_state(u0, v0, step=3, dt=4e-5)
    ob.step(1, force=force)
    uo, vo = ob.get_state()
    with tl.from_workload(body, precision=64) as gb:
        gb.set_state(u0, v0, step=3, dt=4e-5)
        rep = gb.step(1, force_damping=force)
        ug, vg, step, dt = gb.get_state()
    assert rep["damped_steps"] == force and step == 4
    assert rel(ug - u0, uo - u0) < 1e-10
    assert rel(vg - v0, vo - v0) < 1e-10
    assert dt == pytest.approx(ob.dt, rel=1e-10)


@pytest.mark.parametrize("dim", [2, 3])
def test_trajectory_fp64_random_choice(dim):
    """200 steps from rest with the random-choice rule: the same steps are damped on both sides
    and the states agree to 1e-9 relative."""
    _say(f"trajectory fp64 dim={dim}")
    shape = (36, 6) if dim == 2 else (12, 5, 5)
    body = workloads.small_body(dim, shape, nclamp=3, jitter=0.1, jitter_seed=9, alpha=0.3, seed=11)
    ob = oracle.OracleBody(body)
    nd_o = ob.step(200)
    uo, vo = ob.get_state()
    with tl.from_workload(body, precision=64) as gb:
        rep = gb.step(200)
        ug, vg, step, _ = gb.get_state()
    assert rep["damped_steps"] == nd_o and step == 200
    assert rel(ug, uo) < 1e-9 and rel(vg, vo) < 1e-9


def test_relax_until_matches_oracle_fp64():
    _say("relax_until fp64 small cantilever")
    body = workloads.c1_cantilever_2d()
    ob = oracle.OracleBody(body)
    ro = ob.relax(1e-3, 20000)
    with tl.from_workload(body, precision=64) as gb:
        rg = gb.relax_until(1e-3, 20000)
        ug = gb.get_displacement()
    assert ro["converged"] and rg["converged"]
    assert rg["steps"] == ro["steps"] and rg["damped_steps"] == ro["damped_steps"]
    assert rg["residual"] == pytest.approx(ro["residual"], rel=1e-8)
    assert rel(ug, ob.get_displacement()) < 1e-9


def test_fp32_final_displacement_cantilever():
    """FP32 forces/stress/damping with FP64 displacement: the relaxed cantilever matches the FP64
    oracle within 1e-4 relative L2 at equal step counts."""
    _say("fp32 deep relaxation C1")
    body = workloads.c1_cantilever_2d()
    nsteps = 30000
    ob = oracle.OracleBody(body)
    ob.step(nsteps)
    uo = ob.get_displacement()
    with tl.from_workload(body, precision=32) as gb:
        rep = gb.step(nsteps)
        ug = gb.get_displacement()
    assert ob.residual < 1e-7
    err = rel(ug, uo)
    _say(f"  fp32 rel L2 = {err:.3e}, residual {rep['residual']:.2e}")
    assert err < 1e-4


@pytest.mark.parametrize("dim,shape", [(2, (41, 12)), (3, (14, 6, 7))])
def test_fp32_one_step_close(dim, shape):
    """One forced-damped FP32 step against the FP64 oracle (2D and 3D: the FP32 damping scans of
    both dimensions)."""
    _say(f"fp32 one step {dim}d")
    body = workloads.small_body(dim, shape, nclamp=2, jitter=0.15, jitter_seed=5, model="nh")
    u0, v0 = smooth_state(body, seed=2)
    ob = oracle.OracleBody(body)
    ob.set_state(u0, v0, step=0, dt=4e-5)
    ob.step(1, force=1)
    uo, vo = ob.get_state()
    with tl.from_workload(body, precision=32) as gb:
        gb.set_state(u0, v0, step=0, dt=4e-5)
        gb.step(1, force_damping=1)
        ug, vg, _, _ = gb.get_state()
    assert rel(vg - v0, vo - v0) < 1e-4
    assert rel(ug - u0, uo - u0) < 1e-4


@pytest.mark.parametrize("precision", [32, 64])
def test_gpu_runs_are_deterministic_and_resume_exactly(precision):
    _say(f"determinism fp{precision}")
    body = workloads.small_body(3, (16, 6, 6), nclamp=2, jitter=0.1, alpha=0.5)
    with tl.from_workload(body, precision=precision) as a, tl.from_workload(body, precision=precision) as b:
        a.step(80)
        b.step(40)
        u, v, step, dt = b.get_state()
        b.set_state(u, v, step, dt)
        b.step(40)
        ua, va, _, _ = a.get_state()
        ub, vb, _, _ = b.get_state()
    assert np.array_equal(ua, ub) and np.array_equal(va, vb)


def test_nonfinite_state_is_reported():
    _say("error path: NaN state")
    body = workloads.small_body(2, (12, 5), nclamp=2)
    with tl.from_workload(body, precision=64) as gb:
        u = np.zeros((body.n, 2))
        u[5, 0] = np.nan
        gb.set_state(u, None, 0, 1e-5)
        with pytest.raises(tl.TLSPHError) as ei:
            gb.step(3)
        assert ei.value.code == tl.E_NONFINITE


def test_inverted_particle_is_reported():
    _say("error path: J <= 0")
    body = workloads.small_body(2, (12, 5), nclamp=0, model="nh")
    with tl.from_workload(body, precision=32) as gb:
        u = -2.0 * (body.X0 - body.X0.mean(axis=0))   # F = -I: J = 1 in 2D, so mirror one axis only
        u[:, 1] = 0.0
        gb.set_state(u, None, 0, 1e-6)
        with pytest.raises(tl.TLSPHError) as ei:
            gb.step(1)
        assert ei.value.code == tl.E_NONFINITE


@pytest.mark.parametrize("precision", [64, 32])
def test_divergence_is_reported_at_the_oracles_step(precision):
    """Blow-up detection: with the divergence factor set to 2 (the default is 1e6) an ordinary damped
    body trips the rule after its kinetic energy turns over; the GPU reports TLSPH_E_DIVERGED at the
    oracle's step, with a finite state, and a body with the default factor runs through."""
    _say(f"error path: divergence factor fp{precision}")
    body = workloads.small_body(2, (20, 4), nclamp=2, alpha=0.5, jitter=0.05, jitter_seed=3)
    ob = oracle.OracleBody(body)
    ob.set_divergence(2.0)
    with pytest.raises(oracle.OracleError) as eo:
        ob.step(300)
    assert eo.value.code == oracle.E_DIVERGED
    with tl.from_workload(body, precision=precision) as gb:
        gb.set_divergence(2.0)
        with pytest.raises(tl.TLSPHError) as ei:
            gb.step(300)
        assert ei.value.code == tl.E_DIVERGED and "blew up" in str(ei.value)
        u, v, step, _ = gb.get_state()
        assert step == ob.step_index and np.isfinite(u).all() and np.isfinite(v).all()
    with tl.from_workload(body, precision=precision) as gb:
        assert gb.step(300)["step_index"] == 300


@pytest.mark.parametrize("precision", [32, 64])
def test_two_stage_finish_matches_one_stage(monkeypatch, precision):
    """Bodies with many block partials reduce them in two stages (256 workgroups, then the finish).
    Forcing that on a small body changes only the summation tree of E_k and sum |a|^2: the same
    steps are damped, the displacement is bit-identical (the time step uses the exact maxima), and
    the residual, kinetic energy and force residual agree to rounding."""
    _say(f"two-stage finish fp{precision}")
    body = workloads.small_body(3, (14, 6, 7), nclamp=2, jitter=0.15, jitter_seed=3, alpha=0.3, seed=5)
    out = []
    for two in (False, True):
        if two:
            monkeypatch.setenv("TLSPH_TWO_STAGE_MIN", "0")
        with tl.from_workload(body, precision=precision) as gb:
            rep = gb.relax_until(1e-3, 3000)
            out.append((rep, gb.get_displacement()))
        monkeypatch.delenv("TLSPH_TWO_STAGE_MIN", raising=False)
    (r1, u1), (r2, u2) = out
    assert r1["steps"] == r2["steps"] and r1["damped_steps"] == r2["damped_steps"]
    assert np.array_equal(u1, u2)
    for k in ("residual", "kinetic_energy", "force_residual"):
        assert r2[k] == pytest.approx(r1[k], rel=1e-12, abs=1e-300), k


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("dim,shape,scheme", [(2, (41, 12), "pairwise"), (3, (14, 6, 7), "pairwise"),
                                              (3, (14, 6, 7), "particle")])
def test_compact_damping_neighbourhoods_change_nothing(monkeypatch, precision, dim, shape, scheme):
    """Bodies above 2M particles stage only the neighbourhood slots their cells' damping visits read,
    renumbered compactly (slots rewritten at setup).  Forcing that on a small irregular body must leave
    30 forced-damped steps bit-identical: the arithmetic is the same, only LDS addresses move, and a
    slot left out or misnumbered would read another particle's velocity."""
    _say(f"compact damping neighbourhoods fp{precision} {dim}d {scheme}")
    body = workloads.small_body(dim, shape, nclamp=2, jitter=0.15, jitter_seed=7, model="nh", alpha=0.2)
    body.scheme = scheme
    u0, v0 = smooth_state(body, seed=4)
    out = []
    for compact in (False, True):
        if compact:
            monkeypatch.setenv("TLSPH_DAMP_COMPACT_N", "0")
        with tl.from_workload(body, precision=precision) as gb:
            gb.set_state(u0, v0, step=0, dt=4e-5)
            gb.step(30, force_damping=1)
            out.append(gb.get_state()[:2])
        monkeypatch.delenv("TLSPH_DAMP_COMPACT_N", raising=False)
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("long_bricks", [True, False], ids=["long-bricks", "default-bricks"])
@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("dim,shape", [(2, (41, 12)), (3, (14, 6, 7))])
def test_compact_brick_neighbourhoods_change_nothing(monkeypatch, precision, dim, shape, long_bricks):
    """Bodies above 2M particles stage, in pass B, only the slots its bricks' rows read, at their rank
    (brick maps and compact pass-B slots built at setup; a copy where both passes share one slot
    array).  Forcing that on a small irregular body, in the brick configuration of bodies above 8M
    particles (4-cell FP32 bricks, tiled order, one slot array) and in the default one, must leave 30
    forced-damped steps and the von Mises field bit-identical."""
    _say(f"compact brick neighbourhoods fp{precision} {dim}d")
    body = workloads.small_body(dim, shape, nclamp=2, jitter=0.15, jitter_seed=11, model="nh", alpha=0.2)
    u0, v0 = smooth_state(body, seed=6)
    out = []
    for compact in (False, True):
        if long_bricks:
            monkeypatch.setenv("TLSPH_PASSB_LONG_BRICK_N", "0")
        if compact:
            monkeypatch.setenv("TLSPH_BRICK_COMPACT_N", "0")
        with tl.from_workload(body, precision=precision) as gb:
            cells = gb.debug_bricks()
            gb.set_state(u0, v0, step=0, dt=4e-5)
            gb.step(30, force_damping=1)
            u, v, _, _ = gb.get_state()
            out.append((cells, u, v, gb.get_von_mises()))
        monkeypatch.delenv("TLSPH_BRICK_COMPACT_N", raising=False)
        monkeypatch.delenv("TLSPH_PASSB_LONG_BRICK_N", raising=False)
    (c0, u0_, v0_, vm0), (c1, u1, v1, vm1) = out
    assert c0 == c1
    if long_bricks:
        assert c0[0] == c0[1]     # one brick geometry for both passes
    assert np.array_equal(u0_, u1) and np.array_equal(v0_, v1) and np.array_equal(vm0, vm1)
