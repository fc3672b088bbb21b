"""Seeded synthetic workloads shared by the tests, the smoke check and the bench.

This module holds no arithmetic of the method: it only describes problems
(lattice size, material constants, boundary programs, step counts) as plain
data and draws seeded initial fields with numpy.  Both the oracle and the HIP
library consume these descriptions and derive everything else themselves.

The paper measures on small synthetic lattices only (uniaxial tension and
simple shear on 40x40 nodes, a 160x40 cantilever, Sect. 4); the workloads
below are synthetic stand-ins of the same kind at the sizes the benchmark
configurations name.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Tuple

import numpy as np

SIDES = ("left", "right", "bottom", "top")


@dataclasses.dataclass(frozen=True)
class Side:
    """Boundary program of one lattice side.

    bc: "dirichlet" (prescribed momentum j*), "neumann" (prescribed traction T*)
        or "periodic" (paired with the opposite side; test use).
    kind: time function of the load, evaluated at the step index n:
        zero, const (amp), disp_ramp (a wall displacement amp reached at
        constant speed over t1 steps, then held), linear_ramp (amp*min(n/t1,1)),
        sin2_ramp (amp*sin^2(pi n/(2 t1)) for n<t1, amp after), sin_pulse
        (amp*sin(pi n/t1) for n<t1, 0 after), gauss (amp*exp(-(n-t0)^2/(2 w^2))
        for n<=t1, 0 after), ricker (the Ricker wavelet with s=w, for n<t1).
    """
    bc: str
    kind: str = "zero"
    amp: Tuple[float, float] = (0.0, 0.0)
    t0: float = 0.0
    t1: float = 0.0
    width: float = 0.0


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int
    material: str          # "svk" | "neohooke" | "linear"
    mu: float
    nu: float
    tau: float
    steps: int
    sides: Dict[str, Side]
    rho0: float = 1.0
    dx: float = 1.0
    noise: float = 0.0     # amplitude of uniform noise on u0, in units of dx
    seed: int = 1

    @property
    def nodes(self) -> int:
        return self.nx * self.ny

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)

    def u0(self) -> np.ndarray:
        """Initial displacement [2, ny, nx]: zero plus the seeded uniform noise."""
        if self.noise == 0.0:
            return np.zeros((2, self.ny, self.nx))
        rng = np.random.default_rng(self.seed)
        return rng.uniform(-1.0, 1.0, size=(2, self.ny, self.nx)) * (self.noise * self.dx)


def _free():
    return Side("neumann")


def _clamped():
    return Side("dirichlet")


def tension32() -> Workload:
    """32x32 St. Venant-Kirchhoff uniaxial tension, tau=1: the left edge held,
    the right edge pulled to 20 % stretch (6.4 dx) over 2000 steps then held,
    top and bottom traction-free; u0 = seeded noise of 1e-8; 3000 steps."""
    return Workload("tension32", 32, 32, "svk", mu=0.05, nu=0.3, tau=1.0, steps=3000,
                    sides={"left": _clamped(),
                           "right": Side("dirichlet", "disp_ramp", (6.4, 0.0), t1=2000),
                           "bottom": _free(), "top": _free()},
                    noise=1e-8, seed=1)


def shear128(nu: float, material: str = "neohooke") -> Workload:
    """128x128 neo-Hooke simple shear: bottom clamped, top sheared to gamma=0.5
    (64 dx) over 10000 steps, left and right traction-free; 20000 steps."""
    return Workload(f"shear128_nu{nu}", 128, 128, material, mu=0.05, nu=nu, tau=0.55,
                    steps=20000,
                    sides={"bottom": _clamped(),
                           "top": Side("dirichlet", "disp_ramp", (64.0, 0.0), t1=10000),
                           "left": _free(), "right": _free()})


def beam2048() -> Workload:
    """2048x128 neo-Hooke cantilever: left edge clamped, a Gaussian-in-time
    transverse traction pulse (peak 1e-3 mu, std 200 steps, centred at step
    800, free after step 1600) on the right edge; 50000 steps."""
    mu = 0.02
    return Workload("beam2048x128", 2048, 128, "neohooke", mu=mu, nu=0.3, tau=0.55,
                    steps=50000,
                    sides={"left": _clamped(),
                           "right": Side("neumann", "gauss", (0.0, 1e-3 * mu), t0=800.0,
                                         t1=1600.0, width=200.0),
                           "bottom": _free(), "top": _free()})


def tension_large(n: int = 8192, steps: int = 1000) -> Workload:
    """n x n St. Venant-Kirchhoff uniaxial tension, tau=0.55: the left edge
    held, the right edge moved at 3.2e-3 dx per step for the whole run
    (the 32x32 case's pulling speed), top and bottom traction-free."""
    return Workload(f"tension{n}", n, n, "svk", mu=0.05, nu=0.3, tau=0.55, steps=steps,
                    sides={"left": _clamped(),
                           "right": Side("dirichlet", "disp_ramp", (3.2e-3 * steps, 0.0),
                                         t1=float(steps)),
                           "bottom": _free(), "top": _free()})


# ---- seeded generic fields for parity tests --------------------------------------

def smooth_field(nx: int, ny: int, amp: float, seed: int, modes: int = 3) -> np.ndarray:
    """A smooth random vector field [2, ny, nx]: a few low Fourier modes with
    seeded amplitudes and phases, scaled so that max |grad| is about amp."""
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5)[None, :]
    y = (np.arange(ny) + 0.5)[:, None]
    out = np.zeros((2, ny, nx))
    for c in range(2):
        for _ in range(modes):
            kx = 2 * math.pi * rng.integers(0, 3) / nx
            ky = 2 * math.pi * rng.integers(0, 3) / ny
            a = rng.uniform(-1, 1)
            ph = rng.uniform(0, 2 * math.pi)
            out[c] += a * np.sin(kx * x + ky * y + ph) / max(kx + ky, 2 * math.pi / max(nx, ny))
    g = max(np.abs(np.diff(out, axis=1)).max(), np.abs(np.diff(out, axis=2)).max(), 1e-300)
    return out * (amp / g)


def random_field(nx: int, ny: int, amp: float, seed: int) -> np.ndarray:
    """Seeded uniform noise [2, ny, nx] in [-amp, amp]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(2, ny, nx))
