"""The oracle's shared-memory mode (OpenMP over particles, and over the cells of one colour block in
the damping sweep, the paper's own parallelisation of Sec. 3.4) gives bit-identical results for any
thread count: topology, B0, random-choice trajectories with either damping scheme, the von Mises
output and the error paths."""
import numpy as np
import pytest

import oracle
import workloads


@pytest.fixture
def restore_threads():
    n = oracle.threads()
    yield
    oracle.set_threads(n)


def _run(body, threads, steps):
    oracle.set_threads(threads)
    assert oracle.threads() == threads
    ob = oracle.OracleBody(body)
    topo = ob.topology()
    B0 = ob.get_B0()
    nd = ob.step(steps)
    u, v = ob.get_state()
    vm = ob.von_mises()
    return topo, B0, nd, u, v, vm, ob.kinetic_energy, ob.residual, ob.dt


@pytest.mark.parametrize("dim,shape,scheme", [(3, (14, 9, 8), "pairwise"), (3, (10, 7, 7), "particle"),
                                              (2, (40, 9), "pairwise")])
def test_threads_are_bit_identical_to_serial(dim, shape, scheme, restore_threads):
    body = workloads.small_body(dim, shape, nclamp=3, jitter=0.2, jitter_seed=8, alpha=0.5, seed=3, scheme=scheme)
    ref = _run(body, 1, 60)
    for threads in (2, 5):
        got = _run(body, threads, 60)
        for k in ref[0]:
            assert np.array_equal(got[0][k], ref[0][k]), k
        for a, b in zip(got[1:], ref[1:]):
            assert np.array_equal(np.asarray(a), np.asarray(b))


def test_threaded_error_paths(restore_threads):
    """A singular B0 and an inverted particle are reported the same way by the threaded oracle."""
    oracle.set_threads(4)
    X0 = np.array([[0.0, 0.0], [0.001, 0.0], [0.002, 0.0]])
    with pytest.raises(oracle.OracleError) as e:
        oracle.OracleBody(dim=2, X0=X0, dp=0.001)
    assert e.value.code == oracle.E_SINGULAR
    body = workloads.small_body(2, (12, 5), nclamp=0, model="nh")
    ob = oracle.OracleBody(body)
    u = -2.0 * (body.X0 - body.X0.mean(axis=0))
    u[:, 1] = 0.0
    ob.set_state(u, None, 0, 1e-6)
    with pytest.raises(oracle.OracleError) as e:
        ob.step(1)
    assert e.value.code == oracle.E_NONFINITE
