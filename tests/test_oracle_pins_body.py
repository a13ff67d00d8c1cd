"""Pins of the oracle's step against facts the mathematics fixes: exactness of the corrected
gradient for affine fields (Eq. 9), the discrete divergence on a linear stress field (Eqs. 12-13),
momentum conservation of S_m and S_d, symmetry and first-order consistency of the swept pairwise
damping (Eqs. 20, 25, 37-39), exact Verlet free fall (Eqs. 15-17) and the Euler-Bernoulli
cantilever deflection."""
import math

import numpy as np
import pytest

import oracle
import workloads


def _lame(E, nu):
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


BODIES = [(2, (14, 6), 2, 0.1), (3, (8, 5, 5), 2, 0.1), (3, (6, 6, 6), 0, 0.25)]


@pytest.mark.parametrize("dim,shape,nclamp,jitter", BODIES)
def test_affine_displacement_gives_exact_F_everywhere(dim, shape, nclamp, jitter):
    """Eq. 9 makes the corrected gradient exact for linear fields at every particle, the surface
    included: u = A X + c gives F = I + A."""
    body = workloads.small_body(dim, shape, nclamp=nclamp, jitter=jitter, jitter_seed=4)
    body.clamped[:] = 0
    ob = oracle.OracleBody(body)
    rng = np.random.default_rng(dim)
    A = 0.05 * rng.standard_normal((dim, dim))
    u = body.X0 @ A.T + rng.standard_normal(dim) * 1e-3
    ob.set_state(u=u)
    F = ob.get_F()
    assert np.abs(F - (np.eye(dim) + A)[None]).max() < 1e-12


@pytest.mark.parametrize("dim,shape,nclamp,jitter", BODIES)
def test_rigid_rotation_gives_no_internal_force(dim, shape, nclamp, jitter):
    body = workloads.small_body(dim, shape, nclamp=nclamp, jitter=jitter, jitter_seed=5)
    body.clamped[:] = 0
    ob = oracle.OracleBody(body)
    th = 0.4
    R = np.eye(dim)
    R[0, 0] = R[1, 1] = math.cos(th)
    R[0, 1], R[1, 0] = -math.sin(th), math.sin(th)
    ob.set_state(u=body.X0 @ (R - np.eye(dim)).T)
    assert np.abs(ob.get_F() - R[None]).max() < 1e-12
    a = ob.get_accel()
    scale = body.E / body.rho0 / body.dp
    assert np.abs(a - body.g3()[:dim][None]).max() < 1e-9 * scale


def test_linear_stress_field_gives_exact_divergence():
    """Eq. 12 with T = P B0 on a regular lattice: for u quadratic in X (so the stress is linear in
    X to within the tiny amplitude's square), an interior particle's acceleration is div(sigma)/rho0
    + g.  A wrong factor (the 2 of Eq. 12, V, rho0), a sign, or B0 P in place of P B0 fails here."""
    body = workloads.small_body(3, (12, 12, 12), nclamp=0, model="svk", E=1e6, nu=0.3, g=(0.0, 0.0, 0.0))
    ob = oracle.OracleBody(body)
    lam, mu = _lame(1e6, 0.3)
    eps = 1e-7
    rng = np.random.default_rng(7)
    Q = rng.standard_normal((3, 3, 3))
    Q = 0.5 * (Q + Q.transpose(0, 2, 1))          # u_k = eps/2 Q_kab X_a X_b
    X = body.X0 - body.X0.mean(axis=0)
    u = 0.5 * eps * np.einsum("kab,na,nb->nk", Q, X, X)
    ob.set_state(u=u)
    a = ob.get_accel()
    # grad u_ka = eps Q_kab X_b ; strain e = sym(grad u) ; sigma = lam tr(e) I + 2 mu e
    # div sigma_k = lam d_k tr(e) + mu (lap u_k + d_k div u)
    lap = eps * np.einsum("kaa->k", Q)
    grad_div = eps * np.einsum("aak->k", Q)
    div_sigma = (lam + mu) * grad_div + mu * lap
    expect = div_sigma / body.rho0
    centre = np.argmin(np.linalg.norm(X, axis=1))
    assert np.linalg.norm(a[centre] - expect) < 1e-6 * np.linalg.norm(expect)


@pytest.mark.parametrize("model", ["svk", "nh"])
def test_internal_forces_conserve_momentum(model):
    """Eq. 12 is antisymmetric in (i, j) for a free body, so sum_i m a_i = sum_i m b_i."""
    body = workloads.small_body(3, (7, 5, 6), nclamp=0, jitter=0.2, model=model)
    ob = oracle.OracleBody(body)
    rng = np.random.default_rng(8)
    ob.set_state(u=2e-4 * rng.standard_normal(body.X0.shape))
    a = ob.get_accel()
    internal = a - body.g3()[None, :]
    scale = np.abs(internal).max()
    assert scale > 1.0
    assert np.abs(internal.sum(axis=0)).max() < 1e-10 * scale * len(a)


def _damp_matrix(ob, free_dofs, eta_t, dt, n, dim):
    cols = []
    for q in free_dofs:
        v = np.zeros(n * dim)
        v[q] = 1.0
        ob.set_state(v=v.reshape(n, dim), dt=dt)
        ob.damp(eta_t, dt)
        cols.append(ob.get_state()[1].reshape(-1)[free_dofs])
    return np.array(cols).T


@pytest.mark.parametrize("dim,shape,nclamp,jitter", [(2, (7, 4), 2, 0.15), (3, (4, 3, 3), 1, 0.15)])
def test_swept_damping_is_a_symmetric_contraction(dim, shape, nclamp, jitter):
    """With equal masses every pair operator of Eq. 39 is a symmetric linear map of the velocities.
    The sweep of Eq. 25 nested with Eq. 37 (forward order, then the exact reverse, each D_i a
    forward-then-backward row) is a palindrome of them, so S_d is symmetric; it is a contraction
    (eigenvalues in (0, 1]) and leaves a uniform velocity unchanged on a free body.  Any break of
    the reverse order breaks the symmetry."""
    body = workloads.small_body(dim, shape, nclamp=nclamp, jitter=jitter, jitter_seed=9)
    ob = oracle.OracleBody(body)
    n = body.n
    free = np.nonzero(body.clamped == 0)[0]
    dofs = (free[:, None] * dim + np.arange(dim)[None, :]).reshape(-1)
    S = _damp_matrix(ob, dofs, eta_t=ob.eta * 0.3, dt=5e-5, n=n, dim=dim)
    assert np.abs(S - S.T).max() < 1e-13
    w = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert w.min() > 1e-9 and w.max() <= 1.0 + 1e-12
    assert w.min() < 0.9   # the test viscosity is strong enough to act
    if nclamp == 0:
        assert np.allclose(S @ np.ones(len(dofs)), 1.0, atol=1e-13)


def test_swept_damping_conserves_momentum_and_decays_energy():
    body = workloads.small_body(3, (6, 5, 5), nclamp=0, jitter=0.1)
    ob = oracle.OracleBody(body)
    rng = np.random.default_rng(10)
    v0 = rng.standard_normal((body.n, 3))
    ob.set_state(v=v0)
    ob.damp(ob.eta / 0.2, 5e-5)
    v1 = ob.get_state()[1]
    assert np.abs(v1.sum(axis=0) - v0.sum(axis=0)).max() < 1e-12 * np.abs(v0).sum()
    assert (v1 ** 2).sum() < (v0 ** 2).sum()
    ob.set_state(v=np.tile([0.3, -0.2, 0.1], (body.n, 1)))
    ob.damp(ob.eta / 0.2, 5e-5)
    assert np.allclose(ob.get_state()[1], [0.3, -0.2, 0.1], atol=1e-15)


@pytest.mark.parametrize("dim,shape,nclamp", [(2, (7, 4), 2), (3, (4, 3, 3), 1)])
def test_damping_determinant_counts_pair_visits(dim, shape, nclamp):
    """Each pair operator of Eq. 39 leaves the pair's centre-of-mass velocity alone and multiplies
    the relative velocity by f = m^2 / (m^2 - 2 m B) (free-free) or scales the free velocity by
    m / (m - B) (one end clamped), so det S_d is the product of f^D over all visits.  Nested Strang
    (Eq. 37 inside Eq. 25) visits every unordered pair 8 times (4 from each end) with B taken at
    dt / 4:  log det S_d = 8 D sum_pairs log f(dt / 4)."""
    body = workloads.small_body(dim, shape, nclamp=nclamp, jitter=0.15, jitter_seed=12)
    ob = oracle.OracleBody(body)
    t = ob.topology()
    perm, rp, col = t["perm"], t["row_ptr"], t["col"]
    Xs, cl = body.X0[perm], body.clamped[perm]
    dp = body.dp
    h, V, m = 1.3 * dp, dp ** dim, 1000.0 * dp ** dim
    eta_t, dt = ob.eta * 0.05, 5e-5
    expect = 0.0
    for i in range(body.n):
        for e in range(rp[i], rp[i + 1]):
            j = col[e]
            if j < i or (cl[i] and cl[j]):
                continue
            r = np.linalg.norm(Xs[i] - Xs[j])
            B = eta_t * (dt / 4) * 2 * V * V * oracle.wendland(dim, h, r)[1] / r
            f = m * m / (m * m - 2 * m * B) if not (cl[i] or cl[j]) else m / (m - B)
            expect += 8 * dim * math.log(f)
    free = np.nonzero(body.clamped == 0)[0]
    dofs = (free[:, None] * dim + np.arange(dim)[None, :]).reshape(-1)
    S = _damp_matrix(ob, dofs, eta_t=eta_t, dt=dt, n=body.n, dim=dim)
    sign, logdet = np.linalg.slogdet(S)
    assert sign > 0
    assert logdet == pytest.approx(expect, rel=1e-9)


def test_pair_operator_relative_velocity_factor():
    """Eq. 39 multiplies v_ij by f = m_i m_j / (m_i m_j - (m_i + m_j) B) and keeps m_i v_i + m_j v_j."""
    rng = np.random.default_rng(13)
    mi, mj, B = 1.3, 0.7, -0.4
    f = mi * mj / (mi * mj - (mi + mj) * B)
    vi0, vj0 = rng.standard_normal(3), rng.standard_normal(3)
    vi, vj = vi0.copy(), vj0.copy()
    for k in range(1, 9):
        vi, vj = oracle.pair_op(3, mi, mj, B, 0, 0, vi, vj)
        assert np.allclose(vi - vj, (vi0 - vj0) * f ** k, rtol=1e-13)
        assert np.allclose(mi * vi + mj * vj, mi * vi0 + mj * vj0, rtol=1e-13)


def test_damping_first_order_consistency_with_eq20():
    """For a small step, S_d(dt) v - v = 2 dt (dv/dt)^nu of Eq. 20 with eta_t, up to O(dt^2): every
    unordered pair is visited from both of its ends, 4 visits of dt/4 each (the factor 2)."""
    body = workloads.small_body(2, (9, 6), nclamp=2, jitter=0.1, jitter_seed=3)
    ob = oracle.OracleBody(body)
    t = ob.topology()
    perm, rp, col = t["perm"], t["row_ptr"], t["col"]
    Xs = body.X0[perm]
    cl = body.clamped[perm]
    rng = np.random.default_rng(11)
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
    assert errs[0] / errs[1] > 1.8 and errs[1] / errs[2] > 1.8   # first-order: error ~ dt


def test_free_fall_is_exact_verlet():
    """E = 0: no internal force, so position Verlet integrates u = g t^2 / 2 exactly whatever the
    (varying) dt of Eq. 18, and damping leaves the uniform velocity alone."""
    body = workloads.small_body(3, (5, 4, 4), nclamp=0, E=0.0, g=(0.0, -9.81, 0.0), alpha=1.0)
    ob = oracle.OracleBody(body)
    h = 1.3 * body.dp
    t = 0.0
    for n in range(40):
        dt = ob.dt if n else 0.6 * math.sqrt(h / 9.81)
        vmax = 9.81 * t
        expect_dt = 0.6 * min(h / vmax if vmax > 0 else math.inf, math.sqrt(h / 9.81))
        assert dt == pytest.approx(expect_dt, rel=1e-13)
        ob.step(1)
        t += dt
        u, v = ob.get_state()
        assert np.allclose(u[:, 1], -0.5 * 9.81 * t * t, rtol=1e-12)
        assert np.allclose(v[:, 1], -9.81 * t, rtol=1e-12)
        assert np.abs(u[:, [0, 2]]).max() == 0.0


def test_checkpoint_resume_is_bit_exact():
    body = workloads.small_body(2, (12, 4), nclamp=2, jitter=0.05, alpha=0.5)
    a = oracle.OracleBody(body)
    a.step(60)
    ua, va = a.get_state()
    b = oracle.OracleBody(body)
    b.step(30)
    u, v = b.get_state()
    n, dt = b.step_index, b.dt
    c = oracle.OracleBody(body)
    c.set_state(u, v, step=n, dt=dt)
    c.step(30)
    uc, vc = c.get_state()
    assert np.array_equal(ua, uc) and np.array_equal(va, vc)


def test_residual_window_definition():
    body = workloads.c1_cantilever_2d()
    ob = oracle.OracleBody(body)
    lam, mu = _lame(body.E, body.nu)
    c = math.sqrt((lam + 2 * mu / 3) / body.rho0)
    h = 1.3 * body.dp
    dt0 = 0.6 * min(h / c, math.sqrt(h / 9.81))
    ext = body.X0.max(axis=0) - body.X0.min(axis=0) + body.dp
    Tw = ext.max() ** 2 / (ext.min() * c)
    assert ob.window == math.ceil(Tw / dt0)


@pytest.mark.slow
def test_cantilever_matches_euler_bernoulli():
    """2D cantilever under gravity (plane strain): the tip deflection approaches
    rho g H L^4 / (8 E' I) per unit width, I = H^3 / 12, E' = E / (1 - nu^2).  With 10 particles
    through the thickness the discrete beam is softer than the continuum one (the paper's Sec. 4.1
    resolution study shows the same trend: coarser bodies deflect more), by about 12 % in the linear
    regime (g / 100); at full gravity the geometric stiffening of the large deflection (delta / L ~
    0.27) partly cancels it.  Accept 15 % for both and require the discrete beam to be softer in
    the linear case."""
    for gfac, tol_rel in ((1.0, 0.15), (0.01, 0.15)):
        body = workloads.c1_cantilever_2d(g=9.81 * gfac)
        ob = oracle.OracleBody(body)
        rep = ob.relax(1e-6, 40000)
        assert rep["converged"], rep
        u = ob.get_displacement()
        tip = (body.X0[:, 0] > 0.198) & (np.abs(body.X0[:, 1] - 0.01) < 0.0011)
        delta = -u[tip, 1].mean()
        L, H = 0.2, 0.02
        Ep = body.E / (1 - body.nu ** 2)
        eb = body.rho0 * 9.81 * gfac * H * L ** 4 / (8 * Ep * H ** 3 / 12)
        assert abs(delta - eb) / eb < tol_rel, (gfac, delta, eb)
        if gfac < 1.0:
            assert delta > eb


def test_cantilever_converges_to_timoshenko_under_refinement():
    """The stiffness of the discrete beam, pinned tighter than one resolution can: a 2D plane-strain
    cantilever of aspect 5:1 (H = 0.012 m) in the linear regime (g = 0.0981 m/s^2, St Venant-Kirchhoff,
    E = 1e6 Pa, nu = 0.3) relaxed to a force residual below 1e-6 at 6 and at 12 particles through the
    thickness.  The closed form with shear, Timoshenko's q L^4 / (8 E' I) + q L^2 / (2 kappa G A) per
    unit width (kappa = 5/6, E' = E / (1 - nu^2)), is the continuum limit.  The discrete beam is
    softer and the excess must shrink at least 2.5-fold when dp halves (it does 3.3-fold; 24
    particles give 3.0-fold more, order ~1.7), and the Richardson extrapolation of the two with
    second order must land within 5 % of the closed form (it lands at +2.3 %; with the observed
    order from three resolutions, +0.6 %).  A stiffness factor off by 10 %, a dropped volume or a
    wrong sign in the force fails it."""
    E, nu, rho, g = 1e6, 0.3, 1000.0, 0.0981
    H, L = 0.012, 0.06
    Ep = E / (1 - nu ** 2)
    q = rho * g * H
    tim = q * L ** 4 / (8 * Ep * H ** 3 / 12) + q * L ** 2 / (2 * (5 / 6) * (E / (2 * (1 + nu))) * H)
    deltas = []
    for ny in (6, 12):
        dp = H / ny
        wb = workloads.cantilever(2, (5 * ny, ny), dp, nclamp=4, name=f"beam{5 * ny}x{ny}", model="svk", E=E, nu=nu,
                                  rho0=rho, g=(0.0, -g), beta=1.0, Lc=H, alpha=0.2, seed=0)
        ob = oracle.OracleBody(wb)
        for _ in range(100):
            rep = ob.relax(0.0, 2000)
            if rep["force_residual"] < 1e-6:
                break
        assert rep["force_residual"] < 1e-6, rep
        u = ob.get_displacement()
        free = wb.clamped == 0
        tip = free & (wb.X0[:, 0] > wb.X0[free, 0].max() - 0.5 * dp)
        deltas.append(-u[tip, 1].mean())
    e6, e12 = deltas[0] / tim - 1.0, deltas[1] / tim - 1.0
    assert e6 > e12 > 0.0 and e6 / e12 > 2.5, (e6, e12)
    extrapolated = deltas[1] + (deltas[1] - deltas[0]) / 3.0
    assert abs(extrapolated / tim - 1.0) < 0.05, (deltas, tim)
