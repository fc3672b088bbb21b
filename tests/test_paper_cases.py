"""The paper's experiments as workloads (Sect. 4) and its grid error norms
(Eq. griderror, Eq. gridnorm), checked on the CPU: norms against hand-computed
values, the restriction of fine fields, step counts, the load programs as the
oracle evaluates them, and the symmetry of a small tension run in the oracle."""
import math

import numpy as np
import pytest

import oracle
from paper_2502_00920_amd import paper_cases as PC


def make_oracle(name, material, nu, dx, threads=4):
    nx, ny, sides, p = PC.case(name, material, nu, dx)
    o = oracle.Oracle(nx, ny, mu=p["mu"], nu=p["nu"], tau=p["tau"], material=p["material"], rho0=p["rho0"],
                      dx=p["dx"], threads=threads)
    return PC.configure(o, sides), nx, ny


def test_grid_error_norms_by_hand():
    u = np.ones((2, 2, 2))
    ref = 2.0 * np.ones((2, 2, 2))
    e2, einf = PC.grid_errors(u, ref)
    # |du|_2 = sqrt(8), |ref|_2 = sqrt(32), n = 4 nodes
    assert e2 == pytest.approx(0.25 * math.sqrt(8) / math.sqrt(32), rel=1e-15)
    assert einf == pytest.approx(1.0 / math.sqrt(32), rel=1e-15)
    # the maximum norm takes the larger of the two components at any node
    v = np.zeros((2, 3, 3))
    v[1, 2, 0] = -0.7
    v[0, 1, 1] = 0.5
    assert PC.norm_inf(v) == 0.7
    # the plain errors drop the node count: on a 2 x 2 lattice E2 = rms / 4
    rms, mx = PC.plain_errors(u, ref)
    assert rms == pytest.approx(0.5, rel=1e-15) and mx == pytest.approx(0.5, rel=1e-15)
    assert e2 == pytest.approx(rms / 4, rel=1e-15)


def test_restriction_is_exact_for_linear_fields():
    a, b, c = 0.3, -1.7, 2.9
    for factor, nc in [(2, 5), (4, 3), (8, 2)]:
        nf = nc * factor
        xf = (np.arange(nf) + 0.5) / nf
        xc = (np.arange(nc) + 0.5) / nc
        f = np.stack([a + b * xf[None, :] + c * xf[:, None]] * 2)
        g = np.stack([a + b * xc[None, :] + c * xc[:, None]] * 2)
        assert np.abs(PC.restrict(f, factor) - g).max() < 1e-14


def test_step_counts_and_lattices():
    # mu = rho0 = 1: shear wave speed 1, lattice speed sqrt(3)
    assert PC.time_step(0.025) == pytest.approx(0.025 / math.sqrt(3), rel=1e-15)
    assert PC.time_step(0.1, mu=1.0 / 3.0) == pytest.approx(0.1, rel=1e-15)
    assert PC.steps_for(2.2, 0.025) == 152 and PC.steps_for(2.2, 0.05) == 76
    assert PC.steps_for(2.2, 0.003125) == 1219
    assert PC.steps_for(0.1 * 2, 0.1 / math.sqrt(3) * math.sqrt(3)) == 3  # 3.46 steps
    nx, ny, _, p = PC.case("tension", "svk", 0.2, 0.025)
    assert (nx, ny) == (40, 40) and p["mu"] == 1.0 and p["rho0"] == 1.0 and p["tau"] == 0.55
    assert PC.case("wave", "neohooke", 0.2, 0.025)[:2] == (160, 40)


def test_time_interpolation():
    """Quadratic interpolation over three steps: weights sum to 1, a step time
    takes that step alone, and any quadratic in time comes out exact."""
    for dx in (0.05, 0.025, 0.0125, 0.003125):
        for t in (0.3, 2.2, 2.0):
            n0, w = PC.interpolation_weights(t, dx)
            dt = PC.time_step(dx)
            assert n0 * dt <= t + 1e-12 and t < (n0 + 1) * dt
            assert sum(w) == pytest.approx(1.0, abs=1e-14)
            q = lambda tt: 0.7 - 1.3 * tt + 2.1 * tt * tt
            got = sum(wk * q((n0 + k) * dt) for k, wk in enumerate(w))
            assert got == pytest.approx(q(t), rel=1e-12)
    dt = PC.time_step(0.05)
    n0, w = PC.interpolation_weights(10 * dt, 0.05)
    assert n0 == 10 and w == pytest.approx((1.0, 0.0, 0.0), abs=1e-9)


def test_load_programs_in_time_units():
    """The programs, as the oracle evaluates them at step n, against the paper's
    formulas at t = n dt."""
    dx = 0.025
    dt = PC.time_step(dx)
    o, _, _ = make_oracle("tension", "svk", 0.2, dx)
    for n in (1, 40, 69, 115):
        t = n * dt
        assert o.side_value("top", n)[1] == pytest.approx(0.175 * math.sin(math.pi * t / 4) ** 2, rel=1e-13)
    assert o.side_value("top", 152)[1] == pytest.approx(0.175, rel=1e-14)  # t > 2
    assert o.side_value("bottom", 152)[1] == pytest.approx(-0.175, rel=1e-14)
    o, _, _ = make_oracle("shear", "neohooke", 0.2, dx)
    for n in (1, 40, 69, 115):
        assert o.side_value("top", n)[0] == pytest.approx(0.1 * math.sin(math.pi * n * dt / 2), rel=1e-12)
    assert o.side_value("top", 152)[0] == 0.0
    o, _, _ = make_oracle("wave", "neohooke", 0.2, dx)
    s, alpha = 0.215, 0.15
    for n in (30, 58, 69, 80, 97):
        d2 = (n * dt - 1.0) ** 2
        want = alpha * 2.0 / math.sqrt(3.0 * s * math.sqrt(math.pi)) * (1 - d2 / s) * math.exp(-0.5 * d2 / s)
        assert o.side_value("right", n)[1] == pytest.approx(want, rel=1e-12, abs=1e-15)
    assert o.side_value("right", 139)[1] == 0.0  # free after t = 2 (138.6 steps)


def test_tension_run_is_symmetric():
    """Top and bottom pulled apart, left and right free: u_x is odd in x and even
    in y, u_y even in x and odd in y; the top edge moves up."""
    o, nx, ny = make_oracle("tension", "neohooke", 0.2, 0.05)
    o.init()
    o.step(PC.steps_for(2.2, 0.05))
    u = o.read("u")
    scale = np.abs(u).max()
    assert scale > 0
    assert np.abs(u[0] + u[0][:, ::-1]).max() < 1e-12 * scale
    assert np.abs(u[0] - u[0][::-1, :]).max() < 1e-12 * scale
    assert np.abs(u[1] - u[1][:, ::-1]).max() < 1e-12 * scale
    assert np.abs(u[1] + u[1][::-1, :]).max() < 1e-12 * scale
    assert u[1][-1].mean() > 0 and u[1][0].mean() < 0
