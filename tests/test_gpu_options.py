"""The step's options on the GPU against the oracle, through the C ABI: linear
wall extrapolation, the corner rule, second-order boundary differences and the
printed time order (the multi-pass step), sampled load programs, the device
diagnostics watch, host read-out of every storage format, and checkpoints.

Bars as for the plain step (relative L2 over all nodes and components, and the
largest node error as a fraction of the field's largest value): FP64 1e-12,
FP32 1e-5; 16-bit storage is held to the regression bounds of the plain step.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2502_00920_amd import workloads as W

pytestmark = pytest.mark.gpu

THREADS = min(8, os.cpu_count() or 1)
TOL = {"f64": 1e-12, "f32": 1e-5}
HALF_U = {"f16": 1.5e-3, "bf16": 3e-2}


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    from paper_2502_00920_amd import mclbm
    return mclbm


def print_case(tag):
    print(f"\n[case] {tag}", flush=True)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


def node_err(a, b):
    """Largest node error over all nodes, over the wall rows and columns, and
    over the four corners, each as a fraction of max |b|."""
    scale = np.abs(b).max()
    d = np.abs(a - b).max(axis=0) / (scale if scale > 0 else 1.0)
    edge = np.zeros(d.shape, bool)
    edge[0, :] = edge[-1, :] = edge[:, 0] = edge[:, -1] = True
    return float(d.max()), float(d[edge].max()), float(d[[0, 0, -1, -1], [0, -1, 0, -1]].max())


def check(o, s, precision, fields, tag):
    """relative L2 and node-wise errors of fields against the oracle, within the bar"""
    tol = TOL[precision]
    out = {}
    for f in fields:
        a, b = s.read(f), o.read(f)
        e = (rel(a, b),) + node_err(a, b)
        out[f] = e
        assert max(e) <= tol, (tag, f, e)
    print(tag, {f: " ".join(f"{v:.1e}" for v in e) for f, e in out.items()}, flush=True)
    return out


# wall programs: time-dependent momentum on Dirichlet sides, traction on Neumann sides
def walls(code):
    prog = {
        "left": (("dirichlet", "sin_pulse", (2e-4, -1e-4), 0, 40), ("neumann", "sin2_ramp", (-4e-3, 1e-3), 0, 30)),
        "right": (("dirichlet", "const", (3e-4, 1e-4)), ("neumann", "sin2_ramp", (5e-3, -2e-3), 0, 25)),
        "bottom": (("dirichlet", "linear_ramp", (-1e-4, 2e-4), 0, 30), ("neumann", "const", (1e-3, -3e-3))),
        "top": (("dirichlet", "sin_pulse", (1e-4, 2e-4), 0, 35), ("neumann", "sin_pulse", (2e-3, 4e-3), 0, 45)),
    }
    out = {}
    for side, c in zip(W.SIDES, code):
        out[side] = "periodic" if c == "P" else prog[side][0 if c == "D" else 1]
    return out


def pair(M, nx, ny, sides, *, material, precision="f64", mu=0.05, nu=0.2, tau=0.55, u0=None, j0=None,
         extrap="copy", corner=0, boundary_order=1, order="text", tau_plus=None, threads=THREADS):
    o = oracle.Oracle(nx, ny, mu=mu, nu=nu, tau=tau, material=material, threads=threads, extrap=extrap,
                      corner=corner, boundary_order=boundary_order, order=order, tau_plus=tau_plus)
    s = M.Sim(nx, ny, mu=mu, nu=nu, tau=tau, material=material, precision=precision, extrap=extrap,
              corner=corner, boundary_order=boundary_order, time_levels=order, tau_plus=tau_plus or 0.0)
    for side, spec in sides.items():
        args = (spec,) if isinstance(spec, str) else tuple(spec)
        o.set_side(side, *args)
        s.set_side(side, *args)
    o.init(u0, j0)
    s.init(u0, j0)
    return o, s


def fields_for(precision):
    return ("u", "p", "j", "r", "pi", "s") if precision == "f64" else ("u", "p")


LATTICES = [
    (150, 37, "NNNN", "neohooke"),  # every corner Neumann-Neumann
    (67, 19, "DDNN", "svk"),        # mixed corners
    (129, 33, "NDND", "linear"),
    (100, 20, "PPNN", "neohooke"),  # corner-free strip
    (65, 66, "NNNN", "svk"),        # the right wall on lane 0 of its strip
    (300, 140, "NNDN", "svk"),      # interior and edge waves
]


def run_case(M, nx, ny, code, material, precision, tag, **opts):
    u0 = W.smooth_field(nx, ny, 0.05, seed=nx + 3 * ny)
    j0 = W.random_field(nx, ny, 1e-3, seed=nx * ny + 7)
    o, s = pair(M, nx, ny, walls(code), material=material, precision=precision, u0=u0, j0=j0, **opts)
    for n in (1, 9, 30):
        o.step(n - o.n)
        s.step(n - s.n)
        check(o, s, precision, fields_for(precision), f"{tag} step {n}")


# ---- linear extrapolation to the wall and the corner rule (the fused step) ------------------------

@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("nx,ny,code,material", LATTICES)
def test_linear_extrapolation_parity(M, nx, ny, code, material, precision):
    print_case(f"extrap linear {nx}x{ny} {code} {material} {precision}")
    run_case(M, nx, ny, code, material, precision, "extrap", extrap="linear")


def test_linear_extrapolation_momentum_balance(M):
    """Through the ABI: on an x-periodic strip with Neumann top and bottom the
    linear extrapolation closes the discrete momentum balance, so each step
    changes sum_X sum_q c_q f_q by exactly dt nx (T*_bottom + T*_top) at t_n
    (Sect. 3.3), whatever the state."""
    print_case("extrap linear momentum balance")
    nx, ny, mu = 150, 40, 0.05
    sides = {"left": "periodic", "right": "periodic",
             "bottom": ("neumann", "sin2_ramp", (1e-3, -2e-3), 0, 7),
             "top": ("neumann", "sin_pulse", (-5e-4, 3e-3), 0, 9)}
    s = M.Sim(nx, ny, mu=mu, nu=0.2, tau=0.55, material="svk", extrap="linear")
    for side, spec in sides.items():
        s.set_side(side, *((spec,) if isinstance(spec, str) else spec))
    s.init(W.smooth_field(nx, ny, 0.05, seed=4), W.random_field(nx, ny, 1e-3, seed=5))
    dt = s.dt
    for n in range(6):
        m0 = s.diag()["momentum"]
        g_b = math.sin(math.pi * n / 14.0) ** 2 if n < 7 else 1.0
        g_t = math.sin(math.pi * n / 9.0) if n < 9 else 0.0
        expect = dt * nx * (np.array([1e-3, -2e-3]) * g_b + np.array([-5e-4, 3e-3]) * g_t)
        s.step(1)
        dm = s.diag()["momentum"] - m0
        assert np.abs(dm - expect).max() <= 1e-12 * (1 + np.abs(m0).max()), (n, dm, expect)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("corner", [1, 2])
def test_corner_option_parity(M, corner, precision):
    print_case(f"corner option {corner} {precision}")
    run_case(M, 150, 37, "NNNN", "neohooke", precision, f"corner {corner}", corner=corner)
    run_case(M, 65, 66, "NNNN", "svk", precision, f"corner {corner} linear", corner=corner, extrap="linear")


# ---- the multi-pass step: second-order boundary differences, the printed time order ----------------

MULTIPASS = [
    dict(boundary_order=2),
    dict(order="listing"),
    dict(order="listing", boundary_order=2),
    dict(order="listing", extrap="linear"),
    dict(boundary_order=2, extrap="linear", corner=1),
    dict(boundary_order=2, tau_plus=1.0),
]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("opts", MULTIPASS, ids=lambda d: "-".join(f"{k}={v}" for k, v in d.items()))
@pytest.mark.parametrize("nx,ny,code,material", [LATTICES[0], LATTICES[1], LATTICES[3], LATTICES[5]])
def test_multipass_parity(M, nx, ny, code, material, opts, precision):
    print_case(f"multi-pass {opts} {nx}x{ny} {code} {material} {precision}")
    run_case(M, nx, ny, code, material, precision, "multi-pass", **opts)


@pytest.mark.parametrize("precision", ["f16", "bf16"])
def test_multipass_half_storage(M, precision):
    print_case(f"multi-pass half storage {precision}")
    nx, ny = 150, 37
    u0 = W.smooth_field(nx, ny, 0.05, seed=nx + 3 * ny)
    o, s = pair(M, nx, ny, walls("NNDN"), material="svk", precision=precision, u0=u0, order="listing",
                boundary_order=2)
    o.step(30)
    s.step(30)
    e = rel(s.read("u"), o.read("u"))
    print(f"u {e:.2e}", flush=True)
    assert e <= HALF_U[precision]


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_multipass_tension_case(M, precision):
    """A traction-loaded tension block (Sect. 4.1's load on a 40 x 40 lattice)
    in the printed order and with second-order boundary differences, 120 steps."""
    print_case(f"multi-pass tension 40x40 {precision}")
    sides = {"left": ("neumann", "sin2_ramp", (-0.02, 0.0), 0, 60), "right": ("neumann", "sin2_ramp", (0.02, 0.0), 0, 60),
             "bottom": "neumann", "top": "neumann"}
    for opts in (dict(order="listing"), dict(boundary_order=2)):
        o, s = pair(M, 40, 40, sides, material="svk", precision=precision, mu=1.0, nu=0.25, **opts)
        o.step(120)
        s.step(120)
        check(o, s, precision, ("u", "p"), f"tension {opts}")


def test_multipass_checkpoint_and_timed_steps(M):
    """The printed order holds S and T of the previous level: a checkpoint (device
    or host) carries them, and the loaded simulation continues bitwise; timed
    steps equal plain ones bitwise."""
    print_case("multi-pass checkpoint")
    nx, ny = 90, 41

    def make():
        s = M.Sim(nx, ny, mu=0.05, nu=0.2, tau=0.55, material="svk", time_levels="listing", boundary_order=2)
        for side, spec in walls("NNDN").items():
            s.set_side(side, *((spec,) if isinstance(spec, str) else spec))
        s.init(W.smooth_field(nx, ny, 0.03, seed=2))
        return s

    ref = make()
    ref.step(40)
    for host in (False, True):
        a = make()
        a.step(15)
        buf = a.save(host=host)
        b = make()
        b.load(buf)
        assert b.n == 15
        b.step(25)
        assert np.array_equal(b.read("u"), ref.read("u")) and np.array_equal(b.read("j"), ref.read("j"))
    t = make()
    t.step_timed(40)
    assert np.array_equal(t.read("u"), ref.read("u"))


# ---- sampled load programs -----------------------------------------------------------------

@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_table_program(M, precision):
    """A TABLE program on a Neumann and a Dirichlet side against the oracle with
    the same table; a table holding the linear ramp's samples runs bitwise as
    the linear ramp."""
    print_case(f"table program {precision}")
    nx, ny = 80, 30
    rng = np.random.default_rng(3)
    tab_n = np.cumsum(rng.uniform(-0.1, 0.2, 25))
    tab_d = np.sin(np.arange(40) * 0.2)
    sides = {"left": ("dirichlet", "table", (1e-4, -2e-4), 0, 0, 0, tab_d),
             "right": ("neumann", "table", (2e-3, 1e-3), 0, 0, 0, tab_n),
             "bottom": "neumann", "top": ("neumann", "const", (0.0, 1e-3))}
    o, s = pair(M, nx, ny, sides, material="neohooke", precision=precision)
    o.step(50)
    s.step(50)
    check(o, s, precision, ("u", "p"), "table")
    runs = []
    for spec in (("neumann", "linear_ramp", (2e-3, 1e-3), 0, 16), ("neumann", "table", (2e-3, 1e-3), 0, 0, 0,
                                                                     np.arange(17) / 16.0)):
        t = M.Sim(nx, ny, mu=0.05, nu=0.2, tau=0.55, material="svk", precision=precision)
        t.set_side("right", *spec)
        t.init()
        t.step(30)
        runs.append(t.read("u"))
    assert np.array_equal(runs[0], runs[1])


# ---- the diagnostics watch ------------------------------------------------------------------

def test_diagnostics_watch(M):
    """With diag_every = k, mclbm_step checks the state on the device after every
    k-th step and records the first checked step with values that are not
    finite; a run that stays finite records none.  The watch changes no result."""
    print_case("diagnostics watch")
    w = W.shear128(0.49)  # beyond both CFL bounds: diverges within tens of steps
    k = 7
    a = M.sim_from_workload(w, "f64", diag_every=k)
    a.init()
    a.step(300)
    d = a.diag()
    assert d["nonfinite"] and d["first_bad_step"] > 0 and d["first_bad_step"] % k == 0
    # the first multiple of k at which a twin run (no watch) is not finite
    b = M.sim_from_workload(w, "f64")
    b.init()
    first = None
    for n in range(k, 301, k):
        b.step(k)
        if b.diag()["nonfinite"]:
            first = n
            break
    assert first == d["first_bad_step"], (first, d["first_bad_step"])
    c = M.sim_from_workload(W.shear128(0.25), "f64", diag_every=5)
    e = M.sim_from_workload(W.shear128(0.25), "f64")
    for s in (c, e):
        s.init(W.smooth_field(128, 128, 0.01, seed=4))
        s.step(100)
    assert c.diag()["first_bad_step"] == -1 and e.diag()["first_bad_step"] == -1
    assert np.array_equal(c.read("u"), e.read("u"))


# ---- read-out to host memory in every storage format -----------------------------------------

@pytest.mark.parametrize("precision", ["f64", "f32", "f16", "bf16"])
def test_host_read_leaves_the_state(M, precision):
    """A read to host memory is staged in the idle population buffer, a few
    components at a time (16-bit storage holds 18 B per node, less than the
    32 B of H or P): it equals the device read-out bitwise, and a run that read
    every field to the host between its steps ends bitwise as one that did not."""
    print_case(f"host read {precision}")
    nx, ny = 97, 45
    u0 = W.smooth_field(nx, ny, 0.03, seed=8)
    runs = []
    for read_host in (False, True):
        s = M.Sim(nx, ny, mu=0.05, nu=0.2, tau=0.55, material="svk", precision=precision)
        for side, spec in walls("DNNN").items():
            s.set_side(side, *((spec,) if isinstance(spec, str) else spec))
        s.init(u0)
        s.step(10)
        if read_host:
            for f, fid in M.FIELD.items():
                nc = M.mclbm_field_components(fid)
                host = np.full((nc, ny, nx), np.nan)
                M.mclbm_read(s.handle, fid, host.ctypes.data, 0)
                assert np.array_equal(host, s.read(f)), f
        s.step(10)
        runs.append(s.read("u"))
    assert np.array_equal(runs[0], runs[1])


def test_checkpoint_mismatch_is_refused(M):
    print_case("checkpoint mismatch")
    a = M.Sim(40, 30, mu=0.05, nu=0.2, tau=0.55, material="svk", precision="f32")
    a.init()
    buf = a.save()
    for kw in (dict(precision="f64"), dict(precision="f32", time_levels="listing")):
        b = M.Sim(40, 30, mu=0.05, nu=0.2, tau=0.55, material="svk", **kw)
        with pytest.raises(M.MclbmError) as e:
            b.load(buf)
        assert e.value.code == M.MCLBM_EINVAL
    c = M.Sim(41, 30, mu=0.05, nu=0.2, tau=0.55, material="svk", precision="f32")
    with pytest.raises(M.MclbmError) as e:
        c.load(buf)
    assert e.value.code == M.MCLBM_EINVAL
    with pytest.raises(M.MclbmError) as e:
        a.load(buf[:100])
    assert e.value.code == M.MCLBM_EINVAL


def test_server_runs_the_fused_step_only(M):
    print_case("server refuses multi-pass options")
    sv = M.Server(precision="f32", steps_per_round=4, max_active=4, pool_bytes=64 << 20)
    for kw in (dict(boundary_order=2), dict(time_levels=1)):
        p = M.make_params(64, 64, mu=0.05, nu=0.2, tau=0.55, material="svk", precision="f32", **kw)
        sides = [M.make_side("neumann")] * 4
        out = np.empty((2, 64, 64))
        with pytest.raises(M.MclbmError) as e:
            M.mclbm_server_submit(sv._h, p, sides, None, 10, out.ctypes.data)
        assert e.value.code == M.MCLBM_EINVAL


@pytest.mark.parametrize("precision, n", [("f32", 96), ("f64", 96), ("f16", 96), ("f64", 1600)])
def test_captured_steps_replay(M, precision, n):
    """mclbm_step captured into a HIP graph on the simulation's own stream.  The
    captured launches hold the captured steps' arguments (buffers by step parity,
    the wall values of those steps), so a graph of an even number of steps under
    constant wall programs replays as the same steps run eagerly.  Each of five
    replays is checked bitwise against an eager twin, with the twin's eager steps
    and a synchronisation between replays.  The lattices cover every storage
    format's one-launch step, on few march blocks and on many (FP64 on
    1600 x 1600, 2500 march blocks)."""
    import torch
    print_case(f"captured steps {precision} {n}x{n}")
    st = torch.cuda.Stream()
    sides = {"left": ("dirichlet",), "right": ("neumann", "const", (2e-3, -1e-3)), "bottom": "neumann",
             "top": ("dirichlet", "const", (1e-4, 0.0))}
    u0 = W.smooth_field(n, n, 1e-3, 5)
    sims = []
    for _ in range(2):
        s = M.Sim(n, n, mu=0.05, nu=0.2, tau=0.55, material="svk", precision=precision, stream=st)
        for side, spec in sides.items():
            s.set_side(side, *((spec,) if isinstance(spec, str) else tuple(spec)))
        s.init(u0)
        sims.append(s)
    g_sim, e_sim = sims
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        g_sim.step(4)
    for r in range(5):
        g.replay()
        e_sim.step(4)
        torch.cuda.synchronize()
        ug, ue = g_sim.read("u"), e_sim.read("u")
        assert np.isfinite(ue).all() and np.abs(ue).max() > 0
        assert np.array_equal(ug, ue), (precision, n, r, float(np.abs(ug - ue).max()))
    del g
