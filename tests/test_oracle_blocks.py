"""Pins of the oracle's building blocks against closed forms (no GPU).

Each test fixes one piece of the method against mathematics the paper states or
implies, independently of how the oracle writes it:
  - D2Q9 equilibrium and forcing reproduce their moments (Sect. 3.2, Tab. 1)
  - BGK collision keeps r and Pi and adds dt*S to the momentum (Algorithm 1);
    the two-relaxation-time option relaxes its odd and even moments at its two rates
  - St. Venant-Kirchhoff and neo-Hooke stresses (Sect. 4) against hand-derived
    closed forms for simple shear and uniaxial stress, objectivity, hyperelastic
    energy derivatives and their linearisation
  - the lattice stress Pi(H) cancels the linear-elastic stress at nu = 1/4
"""
import math

import numpy as np
import pytest

import oracle

# Tab. 1, typed here independently of the oracle source
E = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]], float)


def lat(mu, rho0=1.0, dx=1.0):
    cs2 = mu / rho0
    c = math.sqrt(3.0 * cs2)
    return cs2, c, dx / c, c * E


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("mu", [0.05, 0.02, 1.0])
def test_feq_moments(seed, mu):
    cs2, c, dt, cq = lat(mu)
    rng = np.random.default_rng(seed)
    r = rng.normal()
    j = rng.normal(size=2)
    Pi = rng.normal(size=3)  # xx, xy, yy
    f = oracle.feq(cs2, cq, r, j, Pi)
    scale = 1.0 + abs(r) + np.abs(j).max() + np.abs(Pi).max()
    tol = 1e-14 * scale * max(1.0, c * c)
    assert abs(f.sum() - r) < tol
    np.testing.assert_allclose(cq.T @ f, j, atol=tol * c)
    M2 = np.einsum("qa,qb,q->ab", cq, cq, f)
    np.testing.assert_allclose([M2[0, 0], M2[0, 1], M2[1, 1]], Pi, atol=tol * c * c)
    # third moment: the closure Q = cs^2 (j d + j d + j d) of Eq. Qlin
    M3 = np.einsum("qa,qb,qc,q->abc", cq, cq, cq, f)
    d = np.eye(2)
    Q = cs2 * (np.einsum("a,bc->abc", j, d) + np.einsum("b,ac->abc", j, d)
               + np.einsum("c,ab->abc", j, d))
    np.testing.assert_allclose(M3, Q, atol=tol * c ** 3)


@pytest.mark.parametrize("mu", [0.05, 0.3])
def test_psi_moments(mu):
    cs2, c, dt, cq = lat(mu)
    S = np.array([0.37, -1.25])
    p = oracle.psi(cs2, cq, S)
    assert abs(p.sum()) < 1e-15
    np.testing.assert_allclose(cq.T @ p, S, rtol=1e-14)
    M2 = np.einsum("qa,qb,q->ab", cq, cq, p)
    np.testing.assert_allclose(M2, 0.0, atol=1e-15)


@pytest.mark.parametrize("tau", [0.55, 1.0, 1.7])
def test_collision_invariants(tau):
    cs2, c, dt, cq = lat(0.05)
    rng = np.random.default_rng(7)
    f = rng.normal(size=9)
    S = rng.normal(size=2)
    fc, r, j, Pi = oracle.collide(cs2, cq, 1.0 / tau, dt, f, S)
    assert abs(fc.sum() - f.sum()) < 1e-14
    np.testing.assert_allclose(np.einsum("qa,qb,q->ab", cq, cq, fc),
                               np.einsum("qa,qb,q->ab", cq, cq, f), atol=1e-14)
    # the collision adds dt * S to the population momentum
    np.testing.assert_allclose(cq.T @ fc, cq.T @ f + dt * S, atol=1e-13)
    np.testing.assert_allclose(j, cq.T @ f + 0.5 * dt * S, atol=1e-14)
    assert r == pytest.approx(f.sum(), abs=1e-15)


def test_collision_relaxes_to_equilibrium_at_tau_one():
    # tau = 1: the post-collision state is f_eq(r, j, Pi) + (1/2) psi dt
    cs2, c, dt, cq = lat(0.05)
    rng = np.random.default_rng(3)
    f = rng.normal(size=9)
    S = rng.normal(size=2)
    fc, r, j, Pi = oracle.collide(cs2, cq, 1.0, dt, f, S)
    expect = oracle.feq(cs2, cq, r, j, Pi) + 0.5 * dt * oracle.psi(cs2, cq, S)
    np.testing.assert_allclose(fc, expect, atol=1e-14)


def moments34(cq, g):
    """The odd third-order moments (xxy, xyy) and the even fourth-order one (xxyy)."""
    cx, cy = cq[:, 0], cq[:, 1]
    return np.array([np.sum(cx * cx * cy * g), np.sum(cx * cy * cy * g)]), np.sum(cx * cx * cy * cy * g)


def test_trt_collision_with_equal_rates_is_bgk():
    cs2, c, dt, cq = lat(0.05)
    rng = np.random.default_rng(11)
    f = rng.normal(size=9)
    S = rng.normal(size=2)
    for tau in (0.55, 1.0, 1.7):
        a = oracle.collide(cs2, cq, 1.0 / tau, dt, f, S)
        b = oracle.collide_trt(cs2, cq, 1.0 / tau, 1.0 / tau, dt, f, S)
        np.testing.assert_allclose(b[0], a[0], atol=1e-14)
        np.testing.assert_allclose(b[2], a[2], atol=1e-15)


@pytest.mark.parametrize("tau,tau_plus", [(0.55, 1.0), (0.55, 0.7), (1.2, 0.6)])
def test_trt_collision_moments(tau, tau_plus):
    """Two relaxation times: r and Pi are kept and the momentum gains dt S, as in
    BGK; the odd third-order non-equilibrium moments relax by (1 - 1/tau), the
    even fourth-order one by (1 - 1/tau_plus)."""
    cs2, c, dt, cq = lat(0.05)
    rng = np.random.default_rng(5)
    f = rng.normal(size=9)
    S = rng.normal(size=2)
    fc, r, j, Pi = oracle.collide_trt(cs2, cq, 1.0 / tau, 1.0 / tau_plus, dt, f, S)
    assert abs(fc.sum() - f.sum()) < 1e-14
    np.testing.assert_allclose(np.einsum("qa,qb,q->ab", cq, cq, fc),
                               np.einsum("qa,qb,q->ab", cq, cq, f), atol=1e-14)
    np.testing.assert_allclose(cq.T @ fc, cq.T @ f + dt * S, atol=1e-13)
    # without a source the equilibrium of the result is that of f
    fc, r, j, Pi = oracle.collide_trt(cs2, cq, 1.0 / tau, 1.0 / tau_plus, dt, f, np.zeros(2))
    feq = oracle.feq(cs2, cq, r, j, Pi)
    odd_in, even_in = moments34(cq, f - feq)
    odd_out, even_out = moments34(cq, fc - feq)
    np.testing.assert_allclose(odd_out, (1 - 1 / tau) * odd_in, atol=1e-15 * c ** 3)
    assert even_out == pytest.approx((1 - 1 / tau_plus) * even_in, abs=1e-15 * c ** 4)


# ---- material laws, Sect. 4 ----------------------------------------------------

def lam_ps(mu, nu):
    return 2 * mu * nu / (1 - 2 * nu)


def test_plane_strain_lambda():
    assert oracle.plane_strain_lambda(0.05, 0.3) == pytest.approx(0.075, rel=1e-15)
    assert oracle.plane_strain_lambda(0.05, 0.25) == 0.05  # exactly mu at nu = 1/4
    assert oracle.plane_strain_lambda(1.0, 0.0) == 0.0


@pytest.mark.parametrize("gamma", [0.1, 0.5, 1.3])
@pytest.mark.parametrize("nu", [0.0, 0.25, 0.3, 0.45, -0.1])
def test_simple_shear_closed_forms(gamma, nu):
    mu = 0.05
    lam = lam_ps(mu, nu)
    H = [[0.0, gamma], [0.0, 0.0]]
    # neo-Hooke: J = 1 and P = mu * gamma * [[0, 1], [1, 0]] for any nu
    P = oracle.stress_P("neohooke", lam, mu, H)
    np.testing.assert_allclose(P, [[0.0, mu * gamma], [mu * gamma, 0.0]], atol=1e-15)
    # St. Venant-Kirchhoff: k = (1 - nu)/(1 - 2 nu)
    k = (1 - nu) / (1 - 2 * nu)
    P = oracle.stress_P("svk", lam, mu, H)
    expect = [[mu * gamma ** 2 * k, mu * gamma * (1 + gamma ** 2 * k)],
              [mu * gamma, mu * gamma ** 2 * k]]
    np.testing.assert_allclose(P, expect, rtol=1e-14, atol=1e-16)


def test_simple_shear_worked_numbers():
    # gamma = 0.5, mu = 0.05, nu = 0: P = [[0.0125, 0.03125], [0.025, 0.0125]]
    P = oracle.stress_P("svk", 0.0, 0.05, [[0.0, 0.5], [0.0, 0.0]])
    np.testing.assert_allclose(P, [[0.0125, 0.03125], [0.025, 0.0125]], rtol=1e-15)


@pytest.mark.parametrize("l1", [0.8, 1.05, 1.2, 1.5])
@pytest.mark.parametrize("nu", [0.0, 0.2, 0.3])
def test_uniaxial_stress_closed_forms(l1, nu):
    mu = 0.05
    lam = lam_ps(mu, nu)
    # SVK: lateral stretch with zero lateral stress, and the axial stress
    l2 = math.sqrt((1 - nu * l1 ** 2) / (1 - nu))
    P = oracle.stress_P("svk", lam, mu, [[l1 - 1, 0.0], [0.0, l2 - 1]])
    assert P[0, 0] == pytest.approx(mu * l1 * (l1 ** 2 - 1) / (1 - nu), rel=1e-13)
    assert abs(P[1, 1]) < 1e-15 and P[0, 1] == 0 and P[1, 0] == 0
    # neo-Hooke
    l2 = math.sqrt((1 - nu) / (1 - 2 * nu + nu * l1 ** 2))
    P = oracle.stress_P("neohooke", lam, mu, [[l1 - 1, 0.0], [0.0, l2 - 1]])
    expect = mu * (l1 ** 2 - 1) * (1 - nu + nu * l1 ** 2) / (l1 * (1 - 2 * nu + nu * l1 ** 2))
    assert P[0, 0] == pytest.approx(expect, rel=1e-13)
    assert abs(P[1, 1]) < 1e-15


def test_uniaxial_worked_numbers():
    # lambda1 = 1.2, nu = 0.3, mu = 0.05
    mu, nu = 0.05, 0.3
    lam = lam_ps(mu, nu)
    l2 = 0.900793301167683  # SVK lateral stretch
    P = oracle.stress_P("svk", lam, mu, [[0.2, 0.0], [0.0, l2 - 1]])
    assert P[0, 0] == pytest.approx(0.0377142857142857, rel=1e-12)
    assert abs(P[1, 1]) < 1e-12
    l2 = 0.917249232131679  # neo-Hooke lateral stretch
    P = oracle.stress_P("neohooke", lam, mu, [[0.2, 0.0], [0.0, l2 - 1]])
    assert P[0, 0] == pytest.approx(0.0249439102564103, rel=1e-12)
    assert abs(P[1, 1]) < 1e-12


@pytest.mark.parametrize("material", ["svk", "neohooke"])
@pytest.mark.parametrize("theta", [0.1, 0.7, 2.5])
def test_objectivity_rigid_rotation(material, theta):
    R = np.array([[math.cos(theta), -math.sin(theta)], [math.sin(theta), math.cos(theta)]])
    P = oracle.stress_P(material, lam_ps(0.05, 0.3), 0.05, R - np.eye(2))
    np.testing.assert_allclose(P, 0.0, atol=1e-16)


def W_svk(F, lam, mu):
    E = 0.5 * (F.T @ F - np.eye(2))
    return 0.5 * lam * np.trace(E) ** 2 + mu * np.trace(E @ E)


def W_nh(F, lam, mu):
    C = F.T @ F
    J = np.linalg.det(F)
    return 0.5 * mu * (np.trace(C) - 2) - mu * math.log(J) + 0.25 * lam * (J * J - 1 - 2 * math.log(J))


@pytest.mark.parametrize("material,W", [("svk", W_svk), ("neohooke", W_nh)])
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_stress_is_energy_derivative(material, W, seed):
    mu, nu = 0.05, 0.3
    lam = lam_ps(mu, nu)
    rng = np.random.default_rng(seed)
    H = rng.uniform(-0.3, 0.3, size=(2, 2))
    F = np.eye(2) + H
    P = oracle.stress_P(material, lam, mu, H)
    h = 1e-6
    dW = np.zeros((2, 2))
    for a in range(2):
        for b in range(2):
            Fp, Fm = F.copy(), F.copy()
            Fp[a, b] += h
            Fm[a, b] -= h
            dW[a, b] = (W(Fp, lam, mu) - W(Fm, lam, mu)) / (2 * h)
    np.testing.assert_allclose(P, dW, atol=1e-9)
    # balance of angular momentum: P F^T is symmetric
    M = P @ F.T
    assert abs(M[0, 1] - M[1, 0]) < 1e-15


@pytest.mark.parametrize("material", ["svk", "neohooke", "linear"])
def test_linearisation_is_hooke(material):
    mu, nu = 0.05, 0.3
    lam = lam_ps(mu, nu)
    rng = np.random.default_rng(11)
    D = rng.normal(size=(2, 2))
    eps = 1e-7
    dP = (oracle.stress_P(material, lam, mu, eps * D) - oracle.stress_P(material, lam, mu, -eps * D)) / (2 * eps)
    hooke = lam * np.trace(D) * np.eye(2) + mu * (D + D.T)
    np.testing.assert_allclose(dP, hooke, atol=1e-8)


def test_zero_gradient_zero_stress():
    for m in ("svk", "neohooke", "linear"):
        assert np.all(oracle.stress_P(m, 0.075, 0.05, np.zeros((2, 2))) == 0.0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lattice_stress_cancels_hooke_at_quarter(seed):
    # at nu = 1/4 the plane-strain lambda equals mu and the bare moment chain
    # already carries the whole linear-elastic stress: P_lin + Pi(H) = 0 exactly
    mu = 0.05
    lam = oracle.plane_strain_lambda(mu, 0.25)
    H = np.random.default_rng(seed).normal(size=(2, 2))
    T = oracle.stress_P("linear", lam, mu, H) + oracle.lattice_Pi(mu, H)
    assert np.all(T == 0.0)


@pytest.mark.parametrize("material", ["svk", "neohooke"])
@pytest.mark.parametrize("scale", [1e-4, 1e-7, 1e-10])
def test_small_strain_keeps_relative_precision(material, scale):
    """At |H| = scale the stress is Hooke's law to O(scale); a form that cancels
    O(mu) terms to leave an O(mu |H|) result loses ~1e-16/scale instead."""
    mu, nu = 0.05, 0.3
    lam = lam_ps(mu, nu)
    D = np.array([[0.3, -0.7], [1.1, 0.2]])
    P = oracle.stress_P(material, lam, mu, scale * D) / scale
    hooke = lam * np.trace(D) * np.eye(2) + mu * (D + D.T)
    assert np.abs(P - hooke).max() <= 5 * scale * mu + 1e-14 * mu
