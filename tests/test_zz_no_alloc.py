"""mclbm_diag_noalloc (the diagnostics with their partial sums in the library's
fixed device array, for callers that cannot allocate) against mclbm_diag,
through the C ABI: two calls in a row, the second on a smaller lattice, and a
state that is not finite."""
import numpy as np
import pytest

from paper_2502_00920_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    from paper_2502_00920_amd import mclbm
    return mclbm


def sim(M, nx, ny, precision, seed):
    s = M.Sim(nx, ny, mu=0.05, nu=0.2, tau=0.55, material="neohooke", precision=precision)
    for side, b in zip(W.SIDES, ("dirichlet", "neumann", "neumann", "neumann")):
        s.set_side(side, b)
    s.init(W.smooth_field(nx, ny, 0.03, seed), W.random_field(nx, ny, 1e-3, seed + 1))
    s.step(7)
    return s


def agree(M, s):
    ref = M.mclbm_diag(s.handle)
    out = M.mclbm_diag_noalloc(s.handle)
    print(f"{s.nx}x{s.ny}: momentum {ref.momentum[0]:.6e} {out.momentum[0]:.6e}, ekin {ref.ekin:.6e} "
          f"{out.ekin:.6e}, max_u {ref.max_u:.6e} {out.max_u:.6e}", flush=True)
    assert out.step == ref.step and out.nonfinite == ref.nonfinite and out.growth == ref.growth
    assert out.cfl_excess == ref.cfl_excess and out.first_bad_step == ref.first_bad_step
    scale = abs(ref.momentum[0]) + abs(ref.momentum[1])
    for k in range(2):
        assert abs(out.momentum[k] - ref.momentum[k]) <= 1e-12 * scale
    assert out.ekin == pytest.approx(ref.ekin, rel=1e-12)
    assert out.max_u == ref.max_u  # a maximum does not depend on the order


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_diagnostics_match(M, precision):
    # a lattice of 16 x 250 = 4000 tiles (more than the array's 1024 partials:
    # blocks take several tiles), then a smaller one of 2 x 12 tiles
    big = sim(M, 1000, 1000, precision, 5)
    agree(M, big)
    small = sim(M, 70, 45, precision, 9)
    agree(M, small)
    del big
    agree(M, small)  # again, after the array held the small lattice's partials


def test_noalloc_diagnostics_flag_nonfinite(M):
    nx, ny = 90, 41
    u0 = W.smooth_field(nx, ny, 0.03, 2)
    u0[1, 20, 44] = np.nan
    s = M.Sim(nx, ny, mu=0.05, nu=0.2, tau=0.55, material="svk")
    s.init(u0)
    ref, out = M.mclbm_diag(s.handle), M.mclbm_diag_noalloc(s.handle)
    assert ref.nonfinite and out.nonfinite
    assert M._lib.mclbm_diag_noalloc(M.C.c_void_p(s.handle), M.C.byref(M.mclbm_diag_out())) == M.MCLBM_EUNSTABLE
