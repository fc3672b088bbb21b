"""Plain FP64 CPU oracle of the moment-chain LBM for hyperelastic solids.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU leg of the
benchmark use it to check the HIP library.  The product path never imports it.

The arithmetic lives in ``mclbm_oracle.c`` (Algorithm 1 of arXiv 2502.00920 as
four separate passes per step, FP64, physical units).  This module only builds
that file with gcc and marshals arguments through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mclbm_oracle.c")
# MCLBM_ORACLE_LIB: another build of the same source (e.g. with other floating-
# point contraction flags), for measuring how rounding order alone moves results
LIB = os.environ.get("MCLBM_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

SIDE = {"left": 0, "right": 1, "bottom": 2, "top": 3}
BC = {"dirichlet": 0, "neumann": 1, "periodic": 2}
MATERIAL = {"svk": 0, "neohooke": 1, "linear": 2}
LOAD = {"zero": 0, "const": 1, "disp_ramp": 2, "linear_ramp": 3, "sin2_ramp": 4,
        "sin_pulse": 5, "gauss": 6, "ricker": 7, "table": 8}
FIELD = {"u": (0, 2), "j": (1, 2), "r": (2, 1), "pi": (3, 3), "h": (4, 4),
         "p": (5, 4), "s": (6, 2)}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, OpenMP on)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = C.CDLL(LIB)
        d, i, i64, vp = C.c_double, C.c_int, C.c_int64, C.c_void_p
        dp = C.POINTER(C.c_double)
        L.orc_create.restype = vp
        L.orc_create.argtypes = [i, i, d, d, d, d, d, i, d, d]
        L.orc_destroy.argtypes = [vp]
        L.orc_dt.restype = d
        L.orc_dt.argtypes = [vp]
        L.orc_stepno.restype = i64
        L.orc_stepno.argtypes = [vp]
        L.orc_set_threads.argtypes = [vp, i]
        L.orc_set_extrap_linear.argtypes = [vp, i]
        L.orc_set_listing_order.argtypes = [vp, i]
        L.orc_set_boundary_order.argtypes = [vp, i]
        L.orc_set_tau_plus.argtypes = [vp, d]
        L.orc_set_corner.argtypes = [vp, i]
        L.orc_set_side_table.restype = i
        L.orc_set_side_table.argtypes = [vp, i, dp, i64]
        L.orc_collide_trt.argtypes = [d, dp, d, d, d, dp, dp, dp, dp, dp, dp]
        L.orc_set_side.restype = i
        L.orc_set_side.argtypes = [vp, i, i, i, d, d, d, d, d]
        L.orc_init.argtypes = [vp, dp, dp]
        L.orc_step.argtypes = [vp, i64]
        L.orc_read.restype = i
        L.orc_read.argtypes = [vp, i, dp]
        L.orc_read_f.argtypes = [vp, dp]
        L.orc_momentum.argtypes = [vp, dp]
        L.orc_set_state.argtypes = [vp, dp, dp]
        L.orc_get_prev.argtypes = [vp, dp, dp]
        L.orc_set_prev.argtypes = [vp, dp, dp]
        L.orc_side_value.argtypes = [vp, i, i64, dp]
        L.orc_diag.argtypes = [vp, dp]
        L.orc_feq.argtypes = [d, dp, d, dp, dp, dp]
        L.orc_psi.argtypes = [d, dp, dp, dp]
        L.orc_collide.argtypes = [d, dp, d, d, dp, dp, dp, dp, dp, dp]
        L.orc_lambda.restype = d
        L.orc_lambda.argtypes = [d, d]
        L.orc_stress_P.argtypes = [i, d, d, dp, dp]
        L.orc_lattice_Pi.argtypes = [d, dp, dp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---- building blocks --------------------------------------------------------

def lattice(mu: float, rho0: float = 1.0, dx: float = 1.0):
    """(cs2, c, dt, cq[9,2]) of the D2Q9 lattice coupled to the material."""
    cs2 = mu / rho0
    c = np.sqrt(3.0) * np.sqrt(cs2)
    e = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]],
                 dtype=np.float64)
    return cs2, c, dx / c, c * e


def feq(cs2, cq, r, j, Pi3):
    out = np.zeros(9)
    lib().orc_feq(cs2, _p(_f64(cq)), r, _p(_f64(j)), _p(_f64(Pi3)), _p(out))
    return out


def psi(cs2, cq, S):
    out = np.zeros(9)
    lib().orc_psi(cs2, _p(_f64(cq)), _p(_f64(S)), _p(out))
    return out


def collide(cs2, cq, omega, dt, f, S):
    """One-node BGK collision with forcing: (f_coll, r, j, Pi(xx, xy, yy))."""
    out, r, j, Pi = np.zeros(9), np.zeros(1), np.zeros(2), np.zeros(3)
    lib().orc_collide(cs2, _p(_f64(cq)), omega, dt, _p(_f64(f)), _p(_f64(S)), _p(out),
                      _p(r), _p(j), _p(Pi))
    return out, float(r[0]), j, Pi


def collide_trt(cs2, cq, omega, omega_plus, dt, f, S):
    """One-node two-relaxation-time collision with forcing (the option):
    (f_coll, r, j, Pi(xx, xy, yy))."""
    out, r, j, Pi = np.zeros(9), np.zeros(1), np.zeros(2), np.zeros(3)
    lib().orc_collide_trt(cs2, _p(_f64(cq)), omega, omega_plus, dt, _p(_f64(f)), _p(_f64(S)), _p(out),
                          _p(r), _p(j), _p(Pi))
    return out, float(r[0]), j, Pi


def plane_strain_lambda(mu, nu):
    return lib().orc_lambda(mu, nu)


def stress_P(material: str, lam: float, mu: float, H) -> np.ndarray:
    """First Piola-Kirchhoff stress for a 2x2 displacement gradient H."""
    Hf = _f64(np.asarray(H, dtype=np.float64).reshape(4))
    out = np.zeros(4)
    lib().orc_stress_P(MATERIAL[material], lam, mu, _p(Hf), _p(out))
    return out.reshape(2, 2)


def lattice_Pi(mu: float, H) -> np.ndarray:
    Hf = _f64(np.asarray(H, dtype=np.float64).reshape(4))
    out = np.zeros(4)
    lib().orc_lattice_Pi(mu, _p(Hf), _p(out))
    return out.reshape(2, 2)


# ---- whole simulation ---------------------------------------------------------

class Oracle:
    """One simulation on the CPU.  Fields come back as [comp, ny, nx] arrays."""

    def __init__(self, nx, ny, *, mu, nu, tau, material="svk", rho0=1.0, dx=1.0,
                 body=(0.0, 0.0), threads=1, extrap="copy", order="text", boundary_order=1,
                 tau_plus=None, corner=0):
        self.nx, self.ny = int(nx), int(ny)
        self._h = lib().orc_create(self.nx, self.ny, dx, rho0, mu, nu, tau,
                                   MATERIAL[material], body[0], body[1])
        if not self._h:
            raise ValueError("oracle rejected the parameters")
        lib().orc_set_threads(self._h, int(threads))
        lib().orc_set_extrap_linear(self._h, 1 if extrap == "linear" else 0)
        lib().orc_set_listing_order(self._h, 1 if order == "listing" else 0)
        if boundary_order not in (1, 2):
            raise ValueError("boundary_order is 1 or 2")
        lib().orc_set_boundary_order(self._h, int(boundary_order))
        if corner not in (0, 1, 2):
            raise ValueError("corner is 0 (mean), 1 (x wall) or 2 (y wall)")
        lib().orc_set_corner(self._h, int(corner))
        if tau_plus is not None:
            if not tau_plus > 0.5:
                raise ValueError("tau_plus must exceed 0.5")
            lib().orc_set_tau_plus(self._h, float(tau_plus))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                lib().orc_destroy(h)
            except TypeError:  # interpreter shutdown: the module's globals are gone
                pass
            self._h = None

    @property
    def dt(self) -> float:
        return lib().orc_dt(self._h)

    @property
    def n(self) -> int:
        return lib().orc_stepno(self._h)

    def set_side(self, side, bc, kind="zero", amp=(0.0, 0.0), t0=0.0, t1=0.0, width=0.0, table=None):
        rc = lib().orc_set_side(self._h, SIDE[side], BC[bc], LOAD[kind], float(amp[0]),
                                float(amp[1]), float(t0), float(t1), float(width))
        if rc != 0:
            raise ValueError(f"oracle rejected side {side}: {bc}/{kind}")
        if kind == "table":
            t = _f64(table).reshape(-1)
            if lib().orc_set_side_table(self._h, SIDE[side], _p(t), t.size) != 0:
                raise ValueError("a table program needs at least one entry")

    def init(self, u0=None, j0=None):
        N = self.nx * self.ny
        u = None if u0 is None else _f64(u0).reshape(2 * N)
        j = None if j0 is None else _f64(j0).reshape(2 * N)
        lib().orc_init(self._h, _p(u) if u is not None else None,
                       _p(j) if j is not None else None)

    def step(self, n: int = 1):
        lib().orc_step(self._h, int(n))

    def read(self, field: str) -> np.ndarray:
        fid, nc = FIELD[field]
        out = np.zeros((nc, self.ny, self.nx))
        if lib().orc_read(self._h, fid, _p(out)) != 0:
            raise ValueError(field)
        return out

    def read_f(self) -> np.ndarray:
        out = np.zeros((9, self.ny, self.nx))
        lib().orc_read_f(self._h, _p(out))
        return out

    def set_state(self, f=None, u=None):
        """Set f(t_n) [9, ny, nx] and u_n [2, ny, nx] directly (None keeps one)."""
        N = self.nx * self.ny
        fa = None if f is None else _f64(f).reshape(9 * N)
        ua = None if u is None else _f64(u).reshape(2 * N)
        lib().orc_set_state(self._h, _p(fa) if fa is not None else None, _p(ua) if ua is not None else None)

    def get_prev(self):
        """The printed order's S_{n-1} [2, ny, nx] and T_{n-1} [4, ny, nx]."""
        Sp, Tp = np.zeros((2, self.ny, self.nx)), np.zeros((4, self.ny, self.nx))
        lib().orc_get_prev(self._h, _p(Sp), _p(Tp))
        return Sp, Tp

    def set_prev(self, Sp=None, Tp=None):
        N = self.nx * self.ny
        sa = None if Sp is None else _f64(Sp).reshape(2 * N)
        ta = None if Tp is None else _f64(Tp).reshape(4 * N)
        lib().orc_set_prev(self._h, _p(sa) if sa is not None else None, _p(ta) if ta is not None else None)

    def momentum(self) -> np.ndarray:
        out = np.zeros(2)
        lib().orc_momentum(self._h, _p(out))
        return out

    def side_value(self, side, n) -> np.ndarray:
        out = np.zeros(2)
        lib().orc_side_value(self._h, SIDE[side], int(n), _p(out))
        return out

    def diag(self) -> dict:
        out = np.zeros(5)
        lib().orc_diag(self._h, _p(out))
        return {"momentum": out[0:2].copy(), "ekin": float(out[2]), "max_u": float(out[3]),
                "nonfinite": bool(out[4])}
