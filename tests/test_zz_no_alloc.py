"""tlsph_get_von_mises_noalloc (the entry point for callers that cannot allocate device memory)
against tlsph_get_von_mises, through the C ABI: two calls in a row on the library's shared scratch
array, the second on a smaller body, each bit-identical to the allocating entry point and within the
von Mises parity bar of the FP64 oracle; the size limit and the J <= 0 report."""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads

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
    rng = np.random.default_rng(seed)
    X = body.X0 - body.X0.min(axis=0)
    L = X.max(axis=0) + body.dp
    D = body.dim
    u = amp * (X @ rng.standard_normal((D, D)).T + np.sin(2 * math.pi * X / L) @ rng.standard_normal((D, D)).T
               * L.max() / 20)
    u[body.clamped == 1] = 0
    return u


@pytest.mark.parametrize("precision", [64, 32])
def test_noalloc_matches_allocating_entry_point(precision):
    bodies = [workloads.small_body(3, (16, 8, 9), nclamp=2, jitter=0.1, model="nh", jitter_seed=3),
              workloads.small_body(3, (9, 5, 6), nclamp=2, jitter=0.1, model="svk", jitter_seed=5)]
    for k, body in enumerate(bodies):           # the second call is on a smaller body
        _say(f"no-alloc von Mises fp{precision}: body {k}, {body.n} particles")
        u = smooth_u(body, seed=k + 1)
        ob = oracle.OracleBody(body)
        ob.set_state(u=u)
        vo = ob.von_mises()
        with tl.from_workload(body, precision=precision) as gb:
            gb.set_state(u, None, step=0)
            ref = gb.get_von_mises()
            got = gb.get_von_mises_noalloc()
            again = gb.get_von_mises_noalloc()
        assert np.array_equal(got, ref), np.abs(got - ref).max()
        assert np.array_equal(again, ref)
        e = np.abs(got - vo).max() / np.abs(vo).max()
        _say(f"  bit-identical to tlsph_get_von_mises; max rel err vs oracle {e:.2e}")
        assert e < (1e-10 if precision == 64 else 1e-4)


def test_noalloc_size_limit_and_inverted_state():
    big = workloads.small_body(2, (1450, 1450), nclamp=0, model="nh")      # 2,102,500 > 2^21 particles
    assert big.n > (1 << 21)
    _say(f"no-alloc limit: {big.n} particles")
    with tl.from_workload(big, precision=32) as gb:
        with pytest.raises(tl.TLSPHError) as ei:
            gb.get_von_mises_noalloc()
        assert ei.value.code == tl.E_LIMIT
    body = workloads.small_body(3, (8, 5, 5), nclamp=0, model="nh")
    with tl.from_workload(body, precision=64) as gb:
        gb.set_state(-2.5 * body.X0, None, step=0)      # F = -1.5 I: J < 0 everywhere
        with pytest.raises(tl.TLSPHError) as e1:
            gb.get_von_mises()
        with pytest.raises(tl.TLSPHError) as e2:
            gb.get_von_mises_noalloc()
        assert e1.value.code == e2.value.code == tl.E_NONFINITE
        assert str(e1.value) == str(e2.value)
