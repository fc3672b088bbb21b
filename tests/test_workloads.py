"""The seeded synthetic inputs against the configurations they stand for (the
lattices, materials, parameters and wall programs of the benchmark workloads,
and the distributions of the serving stream).  No method arithmetic here."""
import math

import numpy as np

from paper_2502_00920_amd import serve as S
from paper_2502_00920_amd import workloads as W


def walls(w):
    return {k: (v.bc, v.kind, v.amp, v.t0, v.t1, v.width) for k, v in w.sides.items()}


def test_tension32():
    w = W.tension32()
    assert (w.nx, w.ny, w.material, w.mu, w.nu, w.tau, w.steps) == (32, 32, "svk", 0.05, 0.3, 1.0, 3000)
    s = walls(w)
    assert s["left"][:2] == ("dirichlet", "zero") and s["bottom"][0] == s["top"][0] == "neumann"
    # the right wall moves 20 % of the 32-node length over 2000 steps: 3.2e-3 dx per step
    assert s["right"][:2] == ("dirichlet", "disp_ramp") and s["right"][2] == (6.4, 0.0) and s["right"][4] == 2000
    assert s["right"][2][0] / s["right"][4] == 3.2e-3
    u0 = w.u0()
    assert u0.shape == (2, 32, 32) and 0 < np.abs(u0).max() <= 1e-8
    np.testing.assert_array_equal(u0, W.tension32().u0())  # seeded


def test_shear128():
    for nu in (0.0, 0.25, 0.45, 0.49):
        w = W.shear128(nu)
        assert (w.nx, w.ny, w.material, w.nu, w.tau, w.steps) == (128, 128, "neohooke", nu, 0.55, 20000)
        s = walls(w)
        # gamma = 0.5 over 10000 steps: the top wall moves 64 dx, 6.4e-3 dx per step
        assert s["top"][:3] == ("dirichlet", "disp_ramp", (64.0, 0.0)) and s["top"][4] == 10000
        assert s["bottom"][:2] == ("dirichlet", "zero") and s["left"][0] == s["right"][0] == "neumann"


def test_beam2048():
    w = W.beam2048()
    assert (w.nx, w.ny, w.material, w.mu, w.nu, w.tau, w.steps) == (2048, 128, "neohooke", 0.02, 0.3, 0.55, 50000)
    bc, kind, amp, t0, t1, width = walls(w)["right"]
    assert (bc, kind, t0, t1, width) == ("neumann", "gauss", 800.0, 1600.0, 200.0)
    assert amp == (0.0, 1e-3 * w.mu)


def test_tension_large():
    w = W.tension_large(8192, 1000)
    assert (w.nx, w.ny, w.material, w.mu, w.nu, w.tau) == (8192, 8192, "svk", 0.05, 0.3, 0.55)
    bc, kind, amp, t0, t1, width = walls(w)["right"]
    assert (bc, kind, t1) == ("dirichlet", "disp_ramp", 1000.0) and amp[0] / t1 == 3.2e-3


def test_seeded_fields():
    a, b = W.smooth_field(40, 30, 0.02, 5), W.smooth_field(40, 30, 0.02, 5)
    np.testing.assert_array_equal(a, b)
    assert a.shape == (2, 30, 40) and not np.array_equal(a, W.smooth_field(40, 30, 0.02, 6))
    g = np.abs(np.diff(a, axis=2)).max()
    assert 0.005 < g < 0.05  # max |grad| about amp
    r = W.random_field(40, 30, 1e-3, 1)
    assert r.shape == (2, 30, 40) and np.abs(r).max() <= 1e-3 and np.abs(r).max() > 9e-4


def test_serving_stream():
    reqs = S.make_requests(2000, seed=0)
    assert reqs == S.make_requests(2000, seed=0)  # seeded
    sides = np.array([r["nx"] for r in reqs])
    assert all(r["nx"] == r["ny"] for r in reqs) and sides.min() >= 64 and sides.max() <= 1024
    # sides log-uniform in [64, 1024]: the median near sqrt(64 * 1024) = 256
    assert 220 < np.median(sides) < 300
    nus = np.array([r["nu"] for r in reqs])
    assert 0.0 <= nus.min() and nus.max() <= 0.45 and abs(nus.mean() - 0.225) < 0.01
    steps = np.array([r["nsteps"] for r in reqs])
    assert steps.min() >= 1000 and steps.max() <= 20000
    mats = [r["material"] for r in reqs]
    assert abs(mats.count("svk") / len(mats) - 0.5) < 0.04
    cases = [r["case"] for r in reqs]
    assert all(abs(cases.count(c) / len(cases) - 1 / 3) < 0.04 for c in ("tension", "shear", "cantilever"))
    for r in reqs:
        assert r["mu"] == 0.05 and r["tau"] == 0.55
        if r["case"] == "tension":  # at most 3.2e-3 dx per step, at most 5 % of the side
            d, t1 = r["sides"]["right"][2][0], r["sides"]["right"][4]
            assert d <= 0.05 * r["nx"] + 1e-12 and d / t1 <= 3.2e-3 + 1e-15
        elif r["case"] == "shear":
            d, t1 = r["sides"]["top"][2][0], r["sides"]["top"][4]
            assert d <= 0.05 * r["nx"] + 1e-12 and d / t1 <= 6.4e-3 + 1e-15
    # mean updates per request of this stream (the serving load's unit)
    assert 1.5e9 < S.lups(reqs) / len(reqs) < 2.3e9
    assert math.isfinite(S.lups(reqs))
