"""Pins of the oracle's von Mises stress (the output of the twisting example, Sec. 4.2) against closed
forms that do not go through its push-forward J^-1 F S F^T: uniaxial stretch (St Venant-Kirchhoff),
equal biaxial stretch in plane strain (tests the out-of-plane stress), simple shear through the
spatial neo-Hookean form sigma = mu/J (b - I) + lambda ln J / J I, hydrostatic and rigid states, and
objectivity; then a whole body under an affine displacement, whose F is exact at every particle."""
import numpy as np
import pytest

import oracle
import workloads

LAM, MU = 1.7, 0.9


def rot3(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    return q if np.linalg.det(q) > 0 else -q


@pytest.mark.parametrize("a", [0.8, 0.97, 1.0, 1.05, 1.3])
def test_uniaxial_stretch_svk(a):
    """F = diag(a, 1, 1): E11 = (a^2 - 1)/2, S11 = (lambda + 2 mu) E11, S22 = S33 = lambda E11;
    sigma11 = a S11, sigma22 = sigma33 = S22 / a, so vm = |sigma11 - sigma22|.  The same in plane
    strain with F = diag(a, 1)."""
    E = 0.5 * (a * a - 1)
    want = abs(a * (LAM + 2 * MU) * E - LAM * E / a)
    for dim in (2, 3):
        F = np.diag([a] + [1.0] * (dim - 1))
        assert oracle.von_mises(dim, "svk", LAM, MU, F) == pytest.approx(want, rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("a", [0.9, 1.02, 1.2])
def test_plane_strain_equal_biaxial_neo_hooke(a):
    """2D F = a I (plane strain): the in-plane stresses are equal and sigma33 = lambda ln J / J
    differs from them by mu (1 - a^-2), which is then the von Mises stress.  The same F in 3D is a
    hydrostatic state with vm = 0."""
    want = MU * abs(1 - a ** -2)
    assert oracle.von_mises(2, "nh", LAM, MU, a * np.eye(2)) == pytest.approx(want, rel=1e-12)
    assert oracle.von_mises(3, "nh", LAM, MU, a * np.eye(3)) < 1e-14
    assert oracle.von_mises(3, "svk", LAM, MU, a * np.eye(3)) < 1e-14


@pytest.mark.parametrize("g", [1e-3, 0.1, 0.7])
def test_simple_shear_neo_hooke(g):
    """F = I + g e1 (x) e2: J = 1, sigma = mu (b - I) with b = F F^T, so sigma11 = mu g^2,
    sigma12 = mu g, the rest 0, and vm = mu g sqrt(g^2 + 3)."""
    F = np.eye(3)
    F[0, 1] = g
    assert oracle.von_mises(3, "nh", LAM, MU, F) == pytest.approx(MU * g * np.sqrt(g * g + 3), rel=1e-12)
    # plane strain: sigma33 = 0 as well (ln J = 0), the same value
    assert oracle.von_mises(2, "nh", LAM, MU, F[:2, :2]) == pytest.approx(MU * g * np.sqrt(g * g + 3), rel=1e-12)


def test_rigid_rotation_and_objectivity():
    rng = np.random.default_rng(5)
    for _ in range(20):
        R = rot3(rng)
        assert oracle.von_mises(3, "nh", LAM, MU, R) < 1e-13
        assert oracle.von_mises(3, "svk", LAM, MU, R) < 1e-13
        F = np.eye(3) + 0.2 * rng.standard_normal((3, 3))
        if np.linalg.det(F) <= 0.2:
            continue
        for model in ("svk", "nh"):
            v0 = oracle.von_mises(3, model, LAM, MU, F)
            assert oracle.von_mises(3, model, LAM, MU, R @ F) == pytest.approx(v0, rel=1e-11)
    th = 0.4
    R2 = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    assert oracle.von_mises(2, "nh", LAM, MU, R2) < 1e-13


def test_inverted_state_is_rejected():
    with pytest.raises(ValueError):
        oracle.von_mises(3, "svk", LAM, MU, np.diag([-1.0, 1.0, 1.0]))


@pytest.mark.parametrize("dim", [2, 3])
def test_body_affine_displacement(dim):
    """u = A X makes F = I + A at every particle (Eq. 9 is exact for affine fields), so every
    particle's von Mises stress is that of F = I + A; u = 0 gives 0."""
    shape = (9, 6) if dim == 2 else (7, 5, 4)
    body = workloads.small_body(dim, shape, nclamp=0, jitter=0.12, jitter_seed=2, model="nh")
    ob = oracle.OracleBody(body)
    assert np.abs(ob.von_mises()).max() == 0.0
    rng = np.random.default_rng(8)
    A = 0.02 * rng.standard_normal((dim, dim))
    ob.set_state(u=body.X0 @ A.T)
    vm = ob.von_mises()
    lam = body.E * body.nu / ((1 + body.nu) * (1 - 2 * body.nu))
    mu = body.E / (2 * (1 + body.nu))
    want = oracle.von_mises(dim, "nh", lam, mu, np.eye(dim) + A)
    assert want > 0
    assert np.abs(vm - want).max() < 1e-8 * want
