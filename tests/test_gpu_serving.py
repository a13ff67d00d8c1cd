"""The request server (continuous batching): every request's result is the same alone, in a mix of
uneven 2D and 3D bodies, and through the single-body entry points; admission respects the memory
budget; a failing request does not disturb the others.

Bodies are small requests of the serving stream (2D 10:1 cantilevers, 3D 10:1:1 cantilevers and
10:10:1 plates, log-uniform E, uniform nu and gravity; the stream's parameter recipe with the
particle count drawn from 1.5k-6k instead of 5k-500k so that each relaxes to 1e-4 in seconds)."""
import sys
import time

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
tl = pytest.importorskip("paper_2103_08932_amd")

BUDGET = 2 << 30


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def small_requests(ids, n_lo=1500, n_hi=6000):
    return [workloads.serving_request(r, n_lo=n_lo, n_hi=n_hi) for r in ids]


def serve(reqs, precision=32, budget=BUDGET, max_slots=16, timeout=300.0):
    """Submits all requests at once; returns [(report, u)] in request order and the stats."""
    out = []
    with tl.Server(budget, max_slots=max_slots, precision=precision) as srv:
        tickets = [srv.submit(wb) for wb in reqs]
        t_end = time.time() + timeout
        for t in tickets:
            rep = None
            while rep is None:
                assert time.time() < t_end, "server did not finish in time"
                rep = srv.wait(t, 1.0)
            u = srv.result(t) if rep["status"] >= 0 else None
            out.append((rep, u))
        stats = srv.stats()
    return out, stats


def single(wb, precision=32):
    with tl.from_workload(wb, precision=precision) as b:
        st = b.relax_until(wb.tol, wb.max_steps)
        return st, b.get_displacement()


def test_server_mix_equals_alone_and_single_body():
    ids = [0, 1, 3, 5, 6, 8]
    reqs = small_requests(ids)
    _say("requests: " + ", ".join(f"{r.name} dim {r.dim} n {r.n}" for r in reqs))
    mix, stats = serve(reqs)
    _say(f"mix stats {stats}")
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    assert stats["peak_active"] >= 2
    for wb, (rep, u) in zip(reqs, mix):
        _say(f"{wb.name}: steps {rep['steps']} damped {rep['damped_steps']} residual {rep['residual']:.3e} "
             f"status {rep['status']}")
        assert rep["status"] == tl.OK and rep["converged"] and rep["residual"] < wb.tol
        (rep1, u1), = serve([wb])[0]
        assert rep1["steps"] == rep["steps"] and rep1["damped_steps"] == rep["damped_steps"]
        assert np.array_equal(u1, u), f"{wb.name}: result differs alone vs in the mix"
        st2 = single(wb)
        rep2, u2 = st2
        assert rep2["steps"] == rep["steps"], (rep2["steps"], rep["steps"])
        assert np.array_equal(u2, u), f"{wb.name}: server result differs from the single-body path"
        dec = tl.damping_decisions(wb.seed, wb.alpha, 0, rep["steps"])
        assert rep["damped_steps"] == int(dec.sum())


def test_server_fp64_matches_single_body():
    reqs = small_requests([2, 9])
    mix, _ = serve(reqs, precision=64)
    for wb, (rep, u) in zip(reqs, mix):
        rep2, u2 = single(wb, precision=64)
        assert rep["status"] == tl.OK and rep2["steps"] == rep["steps"]
        assert np.array_equal(u2, u)


def admission_estimate(dim, n, R=4):
    """The server's admission estimate of a body's device footprint during setup (bytes): state,
    B0, T, the kernel-gradient row sums, row offsets, the damping cell order and setup scratch per particle, 96 (3D) / 26 (2D) CSR entries per particle of
    4 + 3 * 2 + R bytes (column, three halo slots, damping factor), and a fixed overhead."""
    D = dim
    per_particle = 3 * 8 * D + 2 * R * D + 2 * R * D * D + 1 + 8 + 16 + 32 + 8 * D + 1 + 4 + 4 + 4 + 8 + 16 + 4
    compact = (32 * n if n > 1_000_000 else 0) + (36 * n if n > 2_000_000 else 0)   # compact brick / damping maps
    runs = 16 * n                                                                    # brick run descriptors
    return n * per_particle + n * (96 if dim == 3 else 26) * (10 + R) + compact + runs + 64 * 256 + 65536


def test_server_admission_by_memory_budget():
    """A budget of 1.6 times the largest admission estimate admits one or two bodies at a time and
    still serves all of them, with the same results."""
    reqs = small_requests([0, 3, 6, 8, 11, 13])
    budget = int(1.6 * max(admission_estimate(r.dim, r.n) for r in reqs)) + (1 << 20)
    mix, stats = serve(reqs, budget=budget)
    _say(f"budget {budget} stats {stats}")
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    assert stats["pool_peak"] <= budget
    assert stats["peak_active"] <= 3
    alone, _ = serve([reqs[0]])
    assert np.array_equal(alone[0][1], mix[0][1])


def test_server_failed_request_does_not_disturb_others():
    reqs = small_requests([0, 1])
    bad = workloads.small_body(3, (6, 1, 1), nclamp=0)   # a line of particles: B0 is singular
    bad.tol, bad.max_steps = 1e-4, 100
    res, stats = serve([reqs[0], bad, reqs[1]])
    assert res[1][0]["status"] == tl.E_SINGULAR_B0 and res[1][1] is None
    assert "singular" in res[1][0]["error"]
    assert stats["failed"] == 1
    ref, _ = serve(reqs)
    for k, j in ((0, 0), (2, 1)):
        assert res[k][0]["status"] == tl.OK
        assert np.array_equal(res[k][1], ref[j][1])


def test_server_step_limit():
    wb = small_requests([1])[0]
    wb.max_steps = 37
    (rep, u), = serve([wb])[0]
    assert rep["status"] == tl.NOT_CONVERGED and rep["steps"] == 37 and not rep["converged"]
    with tl.from_workload(wb) as b:
        b.step(37)
        assert np.array_equal(b.get_displacement(), u)


def test_server_mixed_dimensions_in_one_group(monkeypatch):
    """One batch group holding 2D and 3D bodies together (they share one launch table while the
    kernels run per dimension): every result equals the body's result alone."""
    monkeypatch.setenv("TLSPH_SERVE_GROUPS", "1")
    reqs = small_requests([0, 1, 2, 5, 9, 12])
    assert {r.dim for r in reqs} == {2, 3}
    mix, stats = serve(reqs)
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    monkeypatch.delenv("TLSPH_SERVE_GROUPS")
    for wb, (rep, u) in zip(reqs, mix):
        (rep1, u1), = serve([wb])[0]
        assert rep["status"] == tl.OK and rep1["steps"] == rep["steps"]
        assert np.array_equal(u1, u), f"{wb.name}: result differs alone vs in a mixed group"


@pytest.mark.parametrize("precision", [32, 64])
def test_server_large_bodies_equal_single_body(precision):
    """Two requests of the stream at its own sizes, a 301,754-particle 3D cantilever and a
    307,825-particle 2D cantilever (requests 10 and 7), served together with two small ones under a
    step limit: each result is bit-identical to the single-body path's over the same steps."""
    big = [workloads.serving_request(10), workloads.serving_request(7)]
    reqs = big + small_requests([0, 1])
    for wb in reqs:
        wb.max_steps = 400
    _say("requests: " + ", ".join(f"{r.name} dim {r.dim} n {r.n}" for r in reqs))
    mix, stats = serve(reqs, precision=precision, budget=4 << 30)
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    for wb, (rep, u) in zip(reqs, mix):
        assert rep["status"] in (tl.OK, tl.NOT_CONVERGED) and rep["steps"] <= 400
        with tl.from_workload(wb, precision=precision) as b:
            b.step(rep["steps"])
            u1 = b.get_displacement()
        _say(f"{wb.name} ({wb.n} particles): {rep['steps']} steps, {rep['damped_steps']} damped, "
             f"max |u| {np.abs(u).max():.3e}")
        assert np.array_equal(u1, u), f"{wb.name}: served result differs from the single-body path"


def test_server_compact_neighbourhoods_equal_single_body(monkeypatch):
    """Bodies above 2M particles keep compact damping neighbourhoods (and compact brick neighbourhoods
    where both pair passes share one brick geometry, as the 2D bodies' do); forcing them on small
    served bodies (2D and 3D, batched launches) must leave every result bit-identical to the
    single-body path with the full neighbourhoods."""
    reqs = small_requests([0, 1, 3, 5])
    assert {r.dim for r in reqs} == {2, 3}
    for wb in reqs:
        wb.max_steps = 300
    full = []
    for wb in reqs:
        with tl.from_workload(wb) as b:
            b.step(300)
            full.append(b.get_displacement())
    monkeypatch.setenv("TLSPH_DAMP_COMPACT_N", "0")
    monkeypatch.setenv("TLSPH_BRICK_COMPACT_N", "0")     # the 2D bodies' bricks (one geometry) too
    mix, stats = serve(reqs)
    monkeypatch.delenv("TLSPH_DAMP_COMPACT_N")
    monkeypatch.delenv("TLSPH_BRICK_COMPACT_N")
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    for wb, (rep, u), u1 in zip(reqs, mix, full):
        assert rep["steps"] == 300
        assert np.array_equal(u, u1), f"{wb.name}: compact served result differs"
