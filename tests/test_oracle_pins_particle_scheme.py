"""Pins of the oracle's particle-by-particle damping scheme (Sec. 3.1, Eqs. 26-35) against what the
mathematics fixes independently of its formulas: exact momentum conservation, dissipation, first-order
consistency with the explicit viscous term of Eq. 20, the backward-Euler limit of a single clamped
neighbour, the equilibration of a pair under infinite viscosity, and the same relaxed equilibrium as
the pairwise scheme."""
import numpy as np
import pytest

import oracle
import workloads


def test_local_update_conserves_momentum_and_dissipates():
    """Momentum exactly, for any coefficients; kinetic energy never grows while every |B_j| <= m / 2.
    (One gradient step does not solve the implicit system exactly: with |B_j| well above m a single
    local update can add energy for adversarial velocities; the swept relaxation of the workloads
    stays dissipative, see the equilibrium test.)"""
    rng = np.random.default_rng(21)
    for nb in (1, 5, 20, 80):
        m = 0.7
        B = -rng.uniform(0.0, 0.5 * m, nb)
        vi0, vj0 = rng.standard_normal(3), rng.standard_normal((nb, 3))
        vi, vj = oracle.pbp_local(3, m, B, np.zeros(nb), vi0, vj0)
        p0 = m * (vi0 + vj0.sum(axis=0))
        assert np.allclose(m * (vi + vj.sum(axis=0)), p0, rtol=0, atol=1e-13 * (1 + np.abs(p0).max()))
        ek0 = (vi0 ** 2).sum() + (vj0 ** 2).sum()
        assert (vi ** 2).sum() + (vj ** 2).sum() <= ek0 * (1 + 1e-14)


def test_local_update_keeps_a_uniform_velocity():
    B = -np.linspace(0.1, 2.0, 12)
    u = np.array([0.3, -0.2, 0.1])
    vi, vj = oracle.pbp_local(3, 1.3, B, np.zeros(12), u, np.tile(u, (12, 1)))
    assert np.array_equal(vi, u) and np.array_equal(vj, np.tile(u, (12, 1)))


@pytest.mark.parametrize("B", [-1e-3, -0.5, -7.0, -1e4])
def test_single_clamped_neighbour_is_backward_euler(B):
    """A wall neighbour (infinite mass, velocity 0): the implicit local equation m dv = B (v + dv)
    has the exact solution v' = m v / (m - B)."""
    m = 1.7
    v = np.array([0.4, -1.1, 2.0])
    vi, vj = oracle.pbp_local(3, m, [B], [1], v, np.zeros((1, 3)))
    assert np.allclose(vi, m * v / (m - B), rtol=1e-14)
    assert np.array_equal(vj, np.zeros((1, 3)))


def test_infinite_viscosity_equilibrates_a_pair():
    """Two free particles under a diverging viscosity end at their common mean velocity, with an
    error falling like (m / B)^2 (B up to 1e4 m, where FP64 cancellation in the neighbour update stays
    far below it)."""
    m = 1.0
    vi0, vj0 = np.array([1.0, -2.0, 0.5]), np.array([-3.0, 0.0, 4.0])
    mean = 0.5 * (vi0 + vj0)
    for B in (-1e2, -1e3, -1e4):
        tol = (m / B) ** 2
        vi, vj = oracle.pbp_local(3, m, [B], [0], vi0, vj0[None, :])
        assert np.abs(vi - mean).max() < tol * np.abs(vi0 - vj0).max()
        assert np.abs(vj[0] - mean).max() < tol * np.abs(vi0 - vj0).max()


def test_sweep_conserves_momentum_and_decays_energy():
    body = workloads.small_body(3, (6, 5, 5), nclamp=0, jitter=0.1, scheme="particle")
    ob = oracle.OracleBody(body)
    rng = np.random.default_rng(22)
    v0 = rng.standard_normal((body.n, 3))
    ob.set_state(v=v0)
    ob.damp(ob.eta / 0.2, 5e-5)
    v1 = ob.get_state()[1]
    assert np.abs(v1.sum(axis=0) - v0.sum(axis=0)).max() < 1e-12 * np.abs(v0).sum()
    assert (v1 ** 2).sum() < (v0 ** 2).sum()


def test_sweep_first_order_consistency_with_eq20():
    """For a small step the sweep of Eq. 25 with the particle-by-particle D_i gives
    S_d(dt) v - v = 2 dt (dv/dt)^nu of Eq. 20 up to O(dt^2): D_i(dt/2) applies particle i's whole row
    to v_i and the reactions to its neighbours, so each unordered pair acts from both of its ends
    in each of the two half sweeps."""
    body = workloads.small_body(2, (9, 6), nclamp=2, jitter=0.1, jitter_seed=3, scheme="particle")
    ob = oracle.OracleBody(body)
    t = ob.topology()
    perm, rp, col = t["perm"], t["row_ptr"], t["col"]
    Xs = body.X0[perm]
    cl = body.clamped[perm]
    rng = np.random.default_rng(23)
    v0 = rng.standard_normal((body.n, 2))
    v0[body.clamped == 1] = 0.0
    vs = v0[perm]
    dp = body.dp
    h, V, m = 1.3 * dp, dp * dp, 1000.0 * dp * dp
    eta_t = 3.0
    rate = np.zeros_like(vs)
    for i in range(body.n):
        if cl[i]:
            continue
        for e in range(rp[i], rp[i + 1]):
            j = col[e]
            r = np.linalg.norm(Xs[i] - Xs[j])
            dW = oracle.wendland(2, h, r)[1]
            rate[i] += 2 * eta_t / m * V * V * (vs[i] - vs[j]) / r * dW
    errs = []
    for dt in (1e-6, 5e-7, 2.5e-7):
        ob.set_state(v=v0)
        ob.damp(eta_t, dt)
        v1 = ob.get_state()[1][perm]
        errs.append(np.abs((v1 - vs) - 2 * dt * rate).max() / np.abs(2 * dt * rate).max())
    assert errs[-1] < 0.02
    assert errs[0] / errs[1] > 1.8 and errs[1] / errs[2] > 1.8


def test_viscous_time_step_limit():
    """Eq. 35 (particle-by-particle scheme only): dt <= 50 h^2 / (nu D) with nu = eta / rho0."""
    body = workloads.small_body(2, (10, 4), nclamp=2, E=1e3, scheme="particle")
    body.beta = 400.0   # a large viscosity so that Eq. 35 binds before Eq. 18
    ob = oracle.OracleBody(body)
    ob.step(1)
    limit = 50 * (1.3 * body.dp) ** 2 / (ob.eta / body.rho0 * 2)
    assert ob.dt == pytest.approx(limit, rel=1e-14)
    body.scheme = "pairwise"
    ob2 = oracle.OracleBody(body)
    ob2.step(1)
    assert ob2.dt > limit


@pytest.mark.slow
def test_both_schemes_relax_to_the_same_equilibrium():
    """The damping only removes kinetic energy, so both schemes relax the 2D cantilever to the same
    static state (the paper's claim for its schemes, Sec. 4.1)."""
    out = {}
    for scheme in ("pairwise", "particle"):
        body = workloads.c1_cantilever_2d(scheme=scheme)
        ob = oracle.OracleBody(body)
        rep = ob.relax(1e-7, 40000)
        assert rep["converged"], (scheme, rep)
        out[scheme] = ob.get_state()[0]
    a, b = out["pairwise"], out["particle"]
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-3
