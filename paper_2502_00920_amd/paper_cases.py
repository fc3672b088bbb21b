"""The paper's numerical experiments (Sect. 4) as workloads, its grid error
norms (Eq. griderror, Eq. gridnorm) and a lattice-refinement study.

The paper states its experiments in dimensionless units and fixes rho0 = 1
and tau = 0.55, but gives no value for the shear modulus.  Here mu = 1: the
shear wave speed sqrt(mu / rho0) is 1, the lattice speed dX / dt = sqrt(3) and
dt = dX / sqrt(3).  (With mu = rho0 / 3, which would put t = 2 and t = 2.2 on
whole steps, the neo-Hooke tension case at nu = -0.1 diverges before t = 2.2,
while the paper reports it as stable.)  The load programs run in steps, so
their break point t = 2 becomes 2 / dt steps, not a whole number; the field at
t = 2.2 is taken by quadratic interpolation in time over the three steps
around it (third order in dt, below the lattice's second-order error).

  uniaxial tension (Sect. 4.1): 1L x 1L; traction alpha sin^2(pi t / 4) for
      t < 2, then alpha, pulling the top and bottom edges apart; left and
      right free; alpha = 0.175 (SVK), 0.35 (neo-Hooke)
  simple shear (Sect. 4.2): 1L x 1L; bottom held; the top moved sideways by
      the momentum alpha sin(pi t / 2) for t < 2, then 0; left and right
      free; alpha = 0.03 (SVK), 0.1 (neo-Hooke)
  bending wave (Sect. 4.3): 4L x 1L beam, left end clamped, top and bottom
      free; on the right end a tangential Ricker traction (alpha = 0.15,
      s = 0.215, t0 = 1) for t < 2, free after; neo-Hooke, nu = 0.2
rho0 = 1 and tau = 0.55 unless given.

No FE reference is available, so the error of a lattice is taken against a
finer lattice of the same case in FP64 (computed here by the HIP path, or
handed in), restricted to the coarse nodes: with cell-centred nodes a coarse node lies half way between fine ones,
so the restriction averages the 2 x 2 fine nodes around it (exact for fields
linear in X) and, over a refinement by 2^k, repeats that k times.

  python -m paper_2502_00920_amd.paper_cases [--case tension] [--material svk]
      [--nu 0.2] [--levels 0.05 0.025 0.0125] [--reference 0.003125]
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np

RHO0 = 1.0
MU = 1.0


def time_step(dx: float, mu: float = MU, rho0: float = RHO0) -> float:
    """dt of a lattice: the D2Q9 lattice speed of sound dX / (sqrt(3) dt) is the
    shear wave speed sqrt(mu / rho0)."""
    return dx / math.sqrt(3.0 * mu / rho0)


def steps_for(t: float, dx: float) -> int:
    """The last whole step at or before time t."""
    return int(math.floor(t / time_step(dx) + 1e-9))


def interpolation_weights(t: float, dx: float):
    """(n0, w): u(t) = sum_k w[k] u_{n0 + k}, quadratic Lagrange interpolation in
    the steps n0, n0 + 1, n0 + 2 with t / dt between the first two."""
    x = t / time_step(dx)
    n0 = max(0, int(math.floor(x + 1e-9)))
    s = x - n0  # in [0, 1)
    return n0, ((s - 1) * (s - 2) / 2, -s * (s - 2), s * (s - 1) / 2)


def case(name: str, material: str, nu: float, dx: float, tau: float = 0.55):
    """(nx, ny, sides, parameters) of one of the paper's experiments."""
    dt = time_step(dx)
    t2 = 2.0 / dt  # the load programs change at t = 2
    if name == "tension":
        alpha = 0.175 if material == "svk" else 0.35
        n = int(round(1.0 / dx))
        # traction on the top edge (outward normal +y) and the bottom edge (-y)
        sides = {"left": "neumann", "right": "neumann",
                 "top": ("neumann", "sin2_ramp", (0.0, alpha), 0.0, t2),
                 "bottom": ("neumann", "sin2_ramp", (0.0, -alpha), 0.0, t2)}
        nx, ny = n, n
    elif name == "shear":
        alpha = 0.03 if material == "svk" else 0.1
        n = int(round(1.0 / dx))
        sides = {"left": "neumann", "right": "neumann", "bottom": ("dirichlet",),
                 "top": ("dirichlet", "sin_pulse", (alpha, 0.0), 0.0, t2)}
        nx, ny = n, n
    elif name == "wave":
        alpha, s, t0 = 0.15, 0.215, 1.0
        nx, ny = int(round(4.0 / dx)), int(round(1.0 / dx))
        # the library's Ricker program runs in steps: width s / dt^2 steps^2,
        # centre t0 / dt, and amplitude alpha / dt (its prefactor carries the
        # width in steps^2)
        sides = {"left": ("dirichlet",), "top": "neumann", "bottom": "neumann",
                 "right": ("neumann", "ricker", (0.0, alpha / dt), t0 / dt, t2, s / dt ** 2)}
    else:
        raise ValueError(name)
    return nx, ny, sides, dict(mu=MU, nu=nu, tau=tau, material=material, rho0=RHO0, dx=dx)


# ---- error norms (Eq. griderror, Eq. gridnorm) --------------------------------------------

def norm2(v) -> float:
    """Grid 2-norm: sqrt of the sum over nodes of v.v; v is [2, ny, nx]."""
    return float(np.sqrt(np.sum(v * v)))


def norm_inf(v) -> float:
    """Grid maximum norm, max over nodes of max(|v1|, |v2|)."""
    return float(np.max(np.abs(v)))


def grid_errors(u, ref):
    """(E2, Einf) of u against ref: E2 = (1/n) |du|_2 / |ref|_2, Einf = |du|_inf / |ref|_2."""
    du = u - ref
    n = u.shape[1] * u.shape[2]
    return norm2(du) / n / norm2(ref), norm_inf(du) / norm2(ref)


def plain_errors(u, ref):
    """(rms, max) relative errors without the node count: |du|_2 / |ref|_2 and
    |du|_inf / |ref|_inf.  In 2D, E2 and Einf equal these times 1/n and about
    1/sqrt(n), so under refinement by 2 their orders exceed these by 2 and 1."""
    du = u - ref
    return norm2(du) / norm2(ref), norm_inf(du) / norm_inf(ref)


def restrict(v, factor: int):
    """A field on a lattice refined by `factor` (a power of 2) at the coarse nodes."""
    while factor > 1:
        v = 0.25 * (v[:, 0::2, 0::2] + v[:, 1::2, 0::2] + v[:, 0::2, 1::2] + v[:, 1::2, 1::2])
        factor //= 2
    return v


# ---- running a case on the GPU ----------------------------------------------------------------

def configure(sim, sides):
    """Set the walls of `sides` on anything with set_side (the HIP path's Sim)."""
    for side, spec in sides.items():
        sim.set_side(side, *((spec,) if isinstance(spec, str) else tuple(spec)))
    return sim


def make_sim(name, material, nu, dx, precision="f64", tau=0.55):
    """A Sim of one case on one lattice, initialised at rest."""
    from . import mclbm
    nx, ny, sides, p = case(name, material, nu, dx, tau)
    s = configure(mclbm.Sim(nx, ny, precision=precision, **p), sides)
    s.init()
    return s


def run(name, material, nu, dx, t=2.2, precision="f64", tau=0.55):
    """u at time t of one case on one lattice (the HIP path), interpolated in
    time, and the diagnostics of the last step run."""
    s = make_sim(name, material, nu, dx, precision, tau)
    n0, w = interpolation_weights(t, dx)
    s.step(n0)
    u = w[0] * s.read("u")
    for k in (1, 2):
        s.step(1)
        u += w[k] * s.read("u")
    return u, s.diag()


def refinement(name, material, nu, levels=(0.05, 0.025, 0.0125), reference=0.003125, t=2.2, tau=0.55,
               reference_u=None):
    """E2 and Einf (and the plain rms / max errors) of each lattice spacing
    against the reference spacing, and the observed orders between successive
    levels.  reference_u, if given, is the reference lattice's u at time t from
    elsewhere; otherwise the HIP path computes it in FP64."""
    if reference_u is None:
        uref, dref = run(name, material, nu, reference, t, "f64", tau)
        ref_finite = not dref["nonfinite"]
    else:
        uref = np.asarray(reference_u, dtype=np.float64)
        ref_finite = bool(np.all(np.isfinite(uref)))
    rows = []
    for dx in levels:
        u, d = run(name, material, nu, dx, t, "f64", tau)
        factor = int(round(dx / reference))
        ref = restrict(uref, factor)
        e2, einf = grid_errors(u, ref)
        erms, emax = plain_errors(u, ref)
        rows.append({"dx": dx, "E2": e2, "Einf": einf, "rms": erms, "max": emax, "finite": not d["nonfinite"]})
    for a, b in zip(rows, rows[1:]):
        r = a["dx"] / b["dx"]
        for k in ("E2", "Einf", "rms", "max"):
            b["order_" + k] = math.log(a[k] / b[k]) / math.log(r)
    return {"case": name, "material": material, "nu": nu, "t": t, "tau": tau, "reference_dx": reference,
            "reference_finite": ref_finite, "levels": rows}


def time_series(name, material, nu, dx, reference, t_end, every=0.5, tau=0.55):
    """E2 and Einf of lattice dx against lattice `reference` at times k * every
    up to t_end (the paper's error history of the bending wave, Sect. 4.3).  The
    steps of the two lattices line up (dt halves with dX), so each sample is taken
    at the coarse step nearest k * every and the matching fine step; the series
    stops at the first sample where either lattice holds a non-finite value."""
    factor = int(round(dx / reference))
    coarse = make_sim(name, material, nu, dx, "f64", tau)
    fine = make_sim(name, material, nu, reference, "f64", tau)
    dt = time_step(dx)
    out, n_done = [], 0
    for k in range(1, int(math.floor(t_end / every + 1e-9)) + 1):
        n = int(round(k * every / dt))
        coarse.step(n - n_done)
        fine.step(factor * (n - n_done))
        n_done = n
        if coarse.diag()["nonfinite"] or fine.diag()["nonfinite"]:
            out.append({"t": n * dt, "finite": False})
            break
        u, ref = coarse.read("u"), restrict(fine.read("u"), factor)
        e2, einf = grid_errors(u, ref)
        out.append({"t": n * dt, "E2": e2, "Einf": einf, "finite": True})
    return {"case": name, "material": material, "nu": nu, "tau": tau, "dx": dx, "reference_dx": reference,
            "samples": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", default="tension", choices=["tension", "shear", "wave"])
    ap.add_argument("--material", default="svk", choices=["svk", "neohooke"])
    ap.add_argument("--nu", type=float, default=0.2)
    ap.add_argument("--tau", type=float, default=0.55)
    ap.add_argument("--t", type=float, default=2.2)
    ap.add_argument("--levels", type=float, nargs="+", default=[0.05, 0.025, 0.0125])
    ap.add_argument("--reference", type=float, default=0.003125)
    a = ap.parse_args()
    print(json.dumps(refinement(a.case, a.material, a.nu, a.levels, a.reference, a.t, a.tau)), flush=True)


if __name__ == "__main__":
    main()
