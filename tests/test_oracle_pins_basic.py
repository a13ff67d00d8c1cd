"""Pins of the oracle's building blocks against facts fixed outside the oracle: numpy's Philox
generator, quadrature of the kernel, finite differences of the strain energies, and the printed
values of the paper."""
import math

import numpy as np
import pytest

import oracle


# ---------------------------------------------------------------------------------- Philox / Eq. 40
def _numpy_block(key, ctr4):
    """numpy's Philox output block for 256-bit counter ``ctr4``: numpy adds one to its counter
    before generating, so start it at ctr4 - 1 (with borrow across the four words)."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(ctr4))
    c = (c - 1) % (1 << 256)
    words = [(c >> (64 * i)) & (2**64 - 1) for i in range(4)]
    return np.random.Philox(key=key, counter=np.array(words, dtype=np.uint64)).random_raw(4)


@pytest.mark.parametrize("key", [0, 1, 5, 2**40 + 17, 2**64 - 1])
@pytest.mark.parametrize("ctr", [0, 1, 2, 1234567, 2**63 + 5])
def test_philox_matches_numpy(key, ctr):
    """Philox4x64-10 of counter c equals numpy's Philox after it steps from counter c - 1
    (numpy increments the counter before each block)."""
    ours = oracle.philox4x64_10([ctr, 0, 0, 0], [key, 0])
    assert np.array_equal(ours, _numpy_block(key, [ctr, 0, 0, 0]))


def test_philox_high_counter_words_and_key():
    rng = np.random.default_rng(3)
    for _ in range(20):
        c = [int(x) for x in rng.integers(1, 2**62, size=4)]
        k = [int(x) for x in rng.integers(0, 2**62, size=2)]
        ours = oracle.philox4x64_10(c, k)
        key = k[0] + (k[1] << 64)
        assert np.array_equal(ours, _numpy_block(key, c))


def test_damped_decision_definition_and_rate():
    """Eq. 40 read as 'damp iff phi < alpha': word 0's top 24 bits against ceil(alpha 2^24)."""
    alpha = 0.2
    thr = math.ceil(alpha * 2**24)
    n = 20000
    hits = 0
    for step in range(n):
        w0 = int(_numpy_block(11, [step, 0, 0, 0])[0])
        expect = (w0 >> 40) < thr
        got = oracle.damped_decision(11, step, alpha)
        assert got == expect
        hits += got
    # binomial: 5 sigma band around alpha n
    sd = math.sqrt(n * alpha * (1 - alpha))
    assert abs(hits - alpha * n) < 5 * sd
    assert all(oracle.damped_decision(3, s, 1.0) for s in range(50))


def test_random_choice_cost_fraction_matches_table(golden):
    """Table 1: the damping time at alpha = 0.2 is about alpha times the alpha = 1 time.  With the
    decision rule the expected fraction of damped steps is alpha."""
    g = golden["random_choice_cost"]
    for a1, a02 in (g["serial"], g["parallel"]):
        assert abs(a02 / a1 - g["alpha"]) < 0.01
    n = 50000
    frac = sum(oracle.damped_decision(1, s, g["alpha"]) for s in range(n)) / n
    assert abs(frac - g["alpha"]) < 0.01


# ---------------------------------------------------------------------------------- Eq. 36
def test_eta_reproduces_printed_values(golden):
    for name in ("eta_ball", "eta_cantilever"):
        e = golden[name]
        val = oracle.eta(e["beta"], e["rho"], e["E"], e["L"])
        digits = e["printed_digits"]
        assert float(f"{val:.{digits}g}") == pytest.approx(e["printed"], rel=1e-12), (name, val)


# ---------------------------------------------------------------------------------- kernel (Sec. 4)
@pytest.mark.parametrize("dim", [2, 3])
def test_wendland_normalisation_by_quadrature(dim):
    """A smoothing kernel integrates to one over its support (radius 2h)."""
    from scipy import integrate
    h = 0.0026
    W = lambda r: oracle.wendland(dim, h, r)[0]
    if dim == 2:
        val = integrate.quad(lambda r: 2 * math.pi * r * W(r), 0, 2 * h, epsabs=0, epsrel=1e-13)[0]
    else:
        val = integrate.quad(lambda r: 4 * math.pi * r * r * W(r), 0, 2 * h, epsabs=0, epsrel=1e-13)[0]
    assert val == pytest.approx(1.0, rel=1e-10)


@pytest.mark.parametrize("dim", [2, 3])
def test_wendland_derivative_by_finite_difference(dim):
    h = 0.0026
    for q in np.linspace(0.05, 1.95, 23):
        r = q * h
        eps = 1e-7 * h
        fd = (oracle.wendland(dim, h, r + eps)[0] - oracle.wendland(dim, h, r - eps)[0]) / (2 * eps)
        assert oracle.wendland(dim, h, r)[1] == pytest.approx(fd, rel=1e-6, abs=1e-9 * abs(fd) + 1e-30)
    assert oracle.wendland(dim, h, 2 * h) == (0.0, 0.0)
    assert oracle.wendland(dim, h, 2.5 * h) == (0.0, 0.0)
    assert oracle.wendland(dim, h, 1.999999 * h)[0] > 0.0


# ---------------------------------------------------------------------------------- Eqs. 4-8
def _energy(model, lam, mu, E):
    """Strain-energy densities: SVK  lam/2 tr(E)^2 + mu tr(E^2);  NH  Eq. 7 with J^2 = det(I + 2E)."""
    D = E.shape[0]
    if model == "svk":
        return 0.5 * lam * np.trace(E) ** 2 + mu * np.trace(E @ E)
    lnJ = 0.5 * math.log(np.linalg.det(np.eye(D) + 2 * E))
    return mu * np.trace(E) - mu * lnJ + 0.5 * lam * lnJ ** 2


@pytest.mark.parametrize("model", ["svk", "nh"])
@pytest.mark.parametrize("dim", [2, 3])
def test_second_piola_is_energy_derivative(model, dim):
    """S = dW/dE (Eq. 8) by central differences in E, and P = F S (Eq. 3)."""
    rng = np.random.default_rng(dim * 10 + (model == "nh"))
    E_mod, nu = 1e6, 0.3
    lam = E_mod * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E_mod / (2 * (1 + nu))
    for _ in range(5):
        F = np.eye(dim) + 0.2 * rng.standard_normal((dim, dim))
        S, P = oracle.stress(dim, model, lam, mu, F)
        Eg = 0.5 * (F.T @ F - np.eye(dim))
        S_fd = np.zeros((dim, dim))
        eps = 1e-6
        for a in range(dim):
            for b in range(dim):
                Ep = Eg.copy(); Ep[a, b] += eps
                Em = Eg.copy(); Em[a, b] -= eps
                S_fd[a, b] = (_energy(model, lam, mu, Ep) - _energy(model, lam, mu, Em)) / (2 * eps)
        S_fd = 0.5 * (S_fd + S_fd.T)
        assert np.allclose(S, S_fd, rtol=1e-6, atol=1e-6 * np.abs(S_fd).max())
        assert np.allclose(P, F @ S, rtol=1e-14, atol=1e-9)


def test_neo_hookean_reduces_to_hooke_at_small_strain():
    lam, mu = 576923.0769, 384615.3846
    rng = np.random.default_rng(4)
    A = 1e-7 * rng.standard_normal((3, 3))
    F = np.eye(3) + A
    S_nh, _ = oracle.stress(3, "nh", lam, mu, F)
    eps = 0.5 * (A + A.T)
    hooke = lam * np.trace(eps) * np.eye(3) + 2 * mu * eps
    assert np.allclose(S_nh, hooke, rtol=1e-5, atol=1e-5 * np.abs(hooke).max())


def test_neo_hookean_rejects_inverted_element():
    with pytest.raises(ValueError):
        oracle.stress(3, "nh", 1.0, 1.0, np.diag([1.0, 1.0, -0.5]))


def test_rigid_rotation_is_stress_free():
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1.0]])
    for model in ("svk", "nh"):
        S, P = oracle.stress(3, model, 2.0, 3.0, R)
        assert np.abs(S).max() < 1e-14 and np.abs(P).max() < 1e-14


# ---------------------------------------------------------------------------------- Eqs. 38-39
def test_pair_op_solves_the_implicit_pair_system():
    """Eq. 39 must satisfy Eq. 38: m_i dv_i = B (v_ij + dv_i - dv_j), m_j dv_j = -B (same)."""
    rng = np.random.default_rng(5)
    for dim in (2, 3):
        for _ in range(50):
            mi, mj = rng.uniform(0.5, 2.0, 2)
            B = -rng.uniform(0, 3)
            vi0, vj0 = rng.standard_normal(dim), rng.standard_normal(dim)
            vi, vj = oracle.pair_op(dim, mi, mj, B, 0, 0, vi0, vj0)
            dvi, dvj = vi - vi0, vj - vj0
            rhs = B * (vi0 - vj0 + dvi - dvj)
            assert np.allclose(mi * dvi, rhs, atol=1e-13)
            assert np.allclose(mj * dvj, -rhs, atol=1e-13)
            assert np.allclose(mi * vi + mj * vj, mi * vi0 + mj * vj0, atol=1e-13)   # momentum


def test_pair_op_clamped_is_infinite_mass_limit():
    rng = np.random.default_rng(6)
    for _ in range(20):
        mi = rng.uniform(0.5, 2)
        B = -rng.uniform(0, 3)
        vi0 = rng.standard_normal(3)
        vj0 = np.zeros(3)
        a_i, a_j = oracle.pair_op(3, mi, 1e12, B, 0, 0, vi0, vj0)
        c_i, c_j = oracle.pair_op(3, mi, 1.0, B, 0, 1, vi0, vj0)
        assert np.allclose(c_i, a_i, rtol=1e-9, atol=1e-12) and np.array_equal(c_j, vj0)
        d_j, d_i = oracle.pair_op(3, 1e12, mi, B, 0, 0, vj0, vi0)
        e_j, e_i = oracle.pair_op(3, 1.0, mi, B, 1, 0, vj0, vi0)
        assert np.allclose(e_i, d_i, rtol=1e-9, atol=1e-12) and np.array_equal(e_j, vj0)
        f_i, f_j = oracle.pair_op(3, 1.0, 1.0, B, 1, 1, vi0, vi0 * 2)
        assert np.array_equal(f_i, vi0) and np.array_equal(f_j, vi0 * 2)
