"""Linear stability of the time step at free walls, on the oracle (no GPU).

With the linear-elastic law and no loads the step is linear in the state
(f(t_n), u_n), so its matrix can be built column by column from the oracle.  On
a lattice periodic in y, translations along y commute with the step: each
wall-parallel wavenumber ky = 2 pi m / ny has its own block of size 11 nx, and
the step's spectral radius is the largest |eigenvalue| over the blocks.  These
tests record what that analysis finds about the scheme of Sect. 3 (BGK, the
anti-bounce-back walls of Eq. abbcon, the source of Eq. source):
  - the bulk is stable at the paper's tau = 0.55;
  - at nu = 1/4 the source vanishes and the scheme is the linear moment chain
    with anti-bounce-back walls: stable at tau = 1 but not at tau = 0.55, where
    a wall mode grows by about 0.26 % per step on a 10-node-wide strip;
  - at nu = 0 the source makes a wave that grazes the wall at the dilatational
    speed c_d grow by 0.6 % per step, the mode behind the long-run divergence of
    runs with free walls.
"""
import math

import numpy as np
import pytest

import oracle

STRIP = {"left": "neumann", "right": "neumann", "bottom": "periodic", "top": "periodic"}
BOX = {"left": "periodic", "right": "periodic", "bottom": "periodic", "top": "periodic"}


def fourier_block(nx, ny, m, sides, **kw):
    """B with step(v(x) e^{i ky y}) = (B v)(x) e^{i ky y}, ky = 2 pi m / ny, for
    the state (f[9], u[2]) per column x."""
    o = oracle.Oracle(nx, ny, **kw)
    for s, b in sides.items():
        o.set_side(s, b)
    o.init()
    ph = np.exp(2j * math.pi * m * np.arange(ny) / ny)
    d = 11 * nx
    B = np.zeros((d, d), complex)
    for k in range(d):
        comp, xi = divmod(k, nx)
        out = []
        for part in (ph.real, ph.imag):
            x = np.zeros((11, ny, nx))
            x[comp, :, xi] = part
            o.set_state(x[:9], x[9:])
            o.step(1)
            out.append(np.concatenate([o.read_f(), o.read("u")]))
        col = ((out[0] + 1j * out[1]) * np.conj(ph)[None, :, None]).sum(axis=1) / ny
        B[:, k] = col.reshape(d)
    return B


def spectral_radius(nx, ny, sides, ms, **kw):
    best = (0.0, None, None)
    for m in ms:
        ev = np.linalg.eigvals(fourier_block(nx, ny, m, sides, **kw))
        i = int(np.argmax(np.abs(ev)))
        if abs(ev[i]) > best[0]:
            best = (float(abs(ev[i])), m, ev[i])
    return best


def test_bulk_is_stable():
    """A periodic box at nu = 0 and tau = 0.55 (no walls): no eigenvalue leaves
    the unit circle beyond the splitting of the step's neutral modes (rigid
    motions, displacements the source does not see) in floating point."""
    rho, m, _ = spectral_radius(12, 16, BOX, range(0, 9), mu=0.05, nu=0.0, tau=0.55, material="linear")
    assert rho <= 1.0 + 1e-5, (rho, m)


@pytest.mark.parametrize("tau, stable", [(1.0, True), (0.55, False)])
def test_anti_bounce_back_walls_without_source(tau, stable):
    """nu = 1/4: P_lin + Pi(H) = 0, the source is zero and the scheme is the
    linear moment chain with the anti-bounce-back walls of Sect. 3.3.  Free walls
    10 nodes apart: stable at tau = 1; at tau = 0.55 an eigenvalue of modulus
    about 1.0026 (ky = 2 pi 3 / 32)."""
    rho, m, lam = spectral_radius(10, 32, STRIP, range(0, 17), mu=0.05, nu=0.25, tau=tau, material="linear")
    if stable:
        assert rho <= 1.0 + 1e-9, (rho, m)
    else:
        assert rho > 1.002 and m == 3, (rho, m)


def test_wall_mode_at_the_dilatational_speed():
    """nu = 0, tau = 0.55, free walls 32 nodes apart, ky = 2 pi 7 / 64: an
    eigenvalue of modulus about 1.0066, a wave along the wall whose phase speed
    |arg lambda| / ky (nodes per step) is the dilatational speed
    c_d / c = sqrt((lambda + 2 mu) / (3 mu)) = sqrt(2/3) within 2 %, and whose
    displacement lies mostly within 8 nodes of the two walls."""
    nx, ny, m = 32, 64, 7
    B = fourier_block(nx, ny, m, STRIP, mu=0.05, nu=0.0, tau=0.55, material="linear")
    ev, V = np.linalg.eig(B)
    i = int(np.argmax(np.abs(ev)))
    assert 1.005 < abs(ev[i]) < 1.008
    ky = 2 * math.pi * m / ny
    speed = abs(np.angle(ev[i])) / ky
    assert speed == pytest.approx(math.sqrt(2.0 / 3.0), rel=0.02)
    u = V[:, i].reshape(11, nx)[9:]
    a = (np.abs(u) ** 2).sum(axis=0)
    near = np.r_[a[:8], a[-8:]].sum() / a.sum()
    assert near > 0.6, near
