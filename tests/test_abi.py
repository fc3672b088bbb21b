"""The C ABI library loads, exports every entry point include/mclbm.h declares,
and rejects bad arguments on the host (no GPU, no kernel launches)."""
import ctypes as C
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mclbm.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mclbm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def M():
    from paper_2502_00920_amd import mclbm
    return mclbm


def test_header_declares_the_api():
    names = declared()
    for n in ["mclbm_plan", "mclbm_create", "mclbm_set_side", "mclbm_init", "mclbm_step",
              "mclbm_read", "mclbm_diag", "mclbm_save", "mclbm_load", "mclbm_destroy",
              "mclbm_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol(M):
    lib = C.CDLL(M.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_shares_torchs_hip_runtime():
    """Imported before torch, the binding still leaves one HIP runtime in the
    process (torch's): a second copy would find no device."""
    code = ("from paper_2502_00920_amd import mclbm\n"
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split()[-1] == "1"


def test_plan_validation(M):
    nbytes, dt = M.mclbm_plan(M.make_params(32, 32, mu=0.05, nu=0.3, tau=1.0))
    assert dt == pytest.approx(1.0 / (3 * 0.05) ** 0.5, rel=1e-15)
    assert nbytes > 2 * 9 * 32 * 64 * 8
    bad = [dict(nx=2), dict(ny=1), dict(tau=0.5), dict(nu=0.5), dict(nu=-1.0), dict(mu=0.0),
           dict(rho0=-1.0), dict(dx=0.0), dict(tau_plus=0.5), dict(tau_plus=-1.0),
           dict(tau_plus=float("nan")), dict(growth_limit=-1.0), dict(growth_limit=float("inf")),
           dict(growth_limit=float("nan"))]
    for b in bad:
        kw = dict(nx=32, ny=32, mu=0.05, nu=0.3, tau=1.0)
        kw.update(b)
        nx, ny = kw.pop("nx"), kw.pop("ny")
        with pytest.raises(M.MclbmError) as e:
            M.mclbm_plan(M.make_params(nx, ny, **kw))
        assert e.value.code == M.MCLBM_EINVAL
    M.mclbm_plan(M.make_params(32, 32, mu=0.05, nu=0.3, tau=1.0, tau_plus=0.8))  # the option is accepted
    M.mclbm_plan(M.make_params(32, 32, mu=0.05, nu=0.3, tau=1.0, growth_limit=2.5))
    # the largest lattices: a displacement buffer (16 B per node of the pitched
    # lattice) must stay below 4 GiB, whatever the population storage
    for n, prec, ok in ((16320, "f32", True), (16384, "f32", False), (16320, "bf16", True),
                        (16320, "f64", True), (16384, "f64", False), (16384, "f16", False)):
        p = M.make_params(n, n, mu=0.05, nu=0.3, tau=0.55, precision=prec)
        if ok:
            assert M.mclbm_plan(p)[0] > 0
        else:
            with pytest.raises(M.MclbmError) as e:
                M.mclbm_plan(p)
            assert e.value.code == M.MCLBM_EINVAL
    # and one lattice row's record of populations (at most 72 B per node of the
    # pitched row) must stay below 4 GiB: a long, short lattice within the
    # displacement bound
    for nx, ok in ((59_652_288, True), (59_652_352, False)):
        p = M.make_params(nx, 3, mu=0.05, nu=0.3, tau=0.55, precision="f16")
        if ok:
            assert M.mclbm_plan(p)[0] > 0
        else:
            with pytest.raises(M.MclbmError) as e:
                M.mclbm_plan(p)
            assert e.value.code == M.MCLBM_EINVAL
    p = M.make_params(32, 32, mu=0.05, nu=0.3, tau=1.0)
    p.material = 7
    with pytest.raises(M.MclbmError):
        M.mclbm_plan(p)
    p = M.make_params(32, 32, mu=0.05, nu=0.3, tau=1.0)
    p.precision = 9
    with pytest.raises(M.MclbmError):
        M.mclbm_plan(p)


def test_arena_scales_with_precision(M):
    b64, _ = M.mclbm_plan(M.make_params(1000, 700, mu=0.05, nu=0.3, tau=0.55, precision="f64"))
    b32, _ = M.mclbm_plan(M.make_params(1000, 700, mu=0.05, nu=0.3, tau=0.55, precision="f32"))
    pitch = 1024
    # two population buffers and two FP64 displacement buffers
    assert b64 >= 2 * 9 * 700 * pitch * 8 + 2 * 2 * 700 * pitch * 8
    assert b32 >= 2 * 9 * 700 * pitch * 4 + 2 * 2 * 700 * pitch * 8
    assert b32 < b64
    b16, _ = M.mclbm_plan(M.make_params(1000, 700, mu=0.05, nu=0.3, tau=0.55, precision="f16"))
    bb16, _ = M.mclbm_plan(M.make_params(1000, 700, mu=0.05, nu=0.3, tau=0.55, precision="bf16"))
    assert b16 == bb16 and b16 >= 2 * 18 * 700 * pitch + 2 * 2 * 700 * pitch * 8 and b16 < b32
    with pytest.raises(M.MclbmError):
        p = M.make_params(100, 100, mu=0.05, nu=0.3, tau=0.55)
        p.precision = 4
        M.mclbm_plan(p)


def test_host_side_errors_without_gpu(M):
    """create only records pointers; misuse is caught before any HIP call."""
    p = M.make_params(16, 16, mu=0.05, nu=0.3, tau=1.0)
    nbytes, _ = M.mclbm_plan(p)
    fake = 1 << 20  # never dereferenced on these paths
    with pytest.raises(M.MclbmError) as e:
        M.mclbm_create(p, fake, nbytes - 1, 0)
    assert e.value.code == M.MCLBM_ETOOSMALL
    with pytest.raises(M.MclbmError) as e:
        M.mclbm_create(p, fake + 8, nbytes, 0)
    assert e.value.code == M.MCLBM_ETOOSMALL
    h = M.mclbm_create(p, fake, nbytes, 0)
    try:
        with pytest.raises(M.MclbmError) as e:
            M.mclbm_step(h, 1)
        assert e.value.code == M.MCLBM_ESTATE
        with pytest.raises(M.MclbmError) as e:
            M.mclbm_step_timed(h, 1)
        assert e.value.code == M.MCLBM_ESTATE
        with pytest.raises(M.MclbmError) as e:
            M.mclbm_step_checked(h, 10, 5)
        assert e.value.code == M.MCLBM_ESTATE
        with pytest.raises(M.MclbmError) as e:
            M.mclbm_read(h, 0, fake, 1)
        assert e.value.code == M.MCLBM_ESTATE
        with pytest.raises(M.MclbmError) as e:
            M.mclbm_set_side(h, 5, M.make_side("neumann"))
        assert e.value.code == M.MCLBM_EINVAL
        with pytest.raises(M.MclbmError) as e:
            M.mclbm_set_side(h, 0, M.make_side("neumann", "disp_ramp", (1, 0), t1=10))
        assert e.value.code == M.MCLBM_EINVAL
        with pytest.raises(M.MclbmError) as e:
            M.mclbm_set_side(h, 0, M.make_side("dirichlet", "sin2_ramp", (1, 0), t1=0))
        assert e.value.code == M.MCLBM_EINVAL
        with pytest.raises(M.MclbmError) as e:
            M.mclbm_set_side(h, 1, M.make_side("neumann", "gauss", (1, 0), t1=10, width=0))
        assert e.value.code == M.MCLBM_EINVAL
        # a periodic side without its partner is refused at init, before any copy
        M.mclbm_set_side(h, 0, M.make_side("periodic"))
        with pytest.raises(M.MclbmError) as e:
            M.mclbm_init(h, None, None, 1)
        assert e.value.code == M.MCLBM_EINVAL
        assert "pair" in M.mclbm_last_error()
        assert M.mclbm_field_components(3) == 3 and M.mclbm_field_components(99) == 0
        assert M.mclbm_stepno(h) == 0
    finally:
        M.mclbm_destroy(h)


def test_copy_argument_errors_without_gpu(M):
    """mclbm_copy rejects bad sizes and pointers before any HIP call; zero bytes is a no-op."""
    fake = 1 << 20
    with pytest.raises(M.MclbmError) as e:
        M.mclbm_copy(fake, fake + 4096, 6, 0)
    assert e.value.code == M.MCLBM_EINVAL
    with pytest.raises(M.MclbmError) as e:
        M.mclbm_copy(fake + 2, fake + 4096, 8, 0)
    assert e.value.code == M.MCLBM_EINVAL
    with pytest.raises(M.MclbmError) as e:
        M.mclbm_copy(None, fake, 8, 0)
    assert e.value.code == M.MCLBM_EINVAL
    M.mclbm_copy(None, None, 0, 0)


def test_server_config_validation(M):
    """The server's configuration is checked on the host."""
    for prec in ("f64", "f32", "f16", "bf16"):
        assert M.mclbm_server_plan(M.mclbm_server_config(M.PRECISION[prec], 32, 64)) > 0
    for bad in [(7, 32, 64), (-1, 32, 64), (M.PRECISION["f32"], 0, 64), (M.PRECISION["f32"], 32, 0),
                (M.PRECISION["f32"], 2000, 64)]:
        with pytest.raises(M.MclbmError) as e:
            M.mclbm_server_plan(M.mclbm_server_config(*bad))
        assert e.value.code == M.MCLBM_EINVAL


def test_product_never_reaches_the_oracle():
    """The oracle is test infrastructure: no module of the package names it, and
    importing every module of the package (the HIP binding included) leaves it
    unloaded."""
    pkg = os.path.join(ROOT, "paper_2502_00920_amd")
    for dirpath, _, files in os.walk(pkg):
        for name in files:
            if name.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                text = open(os.path.join(dirpath, name), errors="replace").read()
                assert "import oracle" not in text and "from oracle" not in text, name
                assert "liboracle" not in text and "mclbm_oracle" not in text, name
    code = ("import sys; import paper_2502_00920_amd.mclbm, paper_2502_00920_amd.serve, "
            "paper_2502_00920_amd.paper_cases, paper_2502_00920_amd.workloads, paper_2502_00920_amd.build; "
            "assert 'oracle' not in sys.modules, 'oracle loaded'; print('clean')")
    p = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert p.returncode == 0 and "clean" in p.stdout, p.stderr[-2000:]


def test_binding_fails_loudly_without_the_library(tmp_path):
    """A copy of the package without libmclbm.so: importing the binding raises
    (there is no CPU fallback to route to)."""
    import shutil
    dst = tmp_path / "paper_2502_00920_amd"
    dst.mkdir()
    for name in os.listdir(os.path.join(ROOT, "paper_2502_00920_amd")):
        if name.endswith(".py"):
            shutil.copy(os.path.join(ROOT, "paper_2502_00920_amd", name), dst / name)
    code = ("import sys; sys.path.insert(0, sys.argv[1])\n"
            "try:\n    import paper_2502_00920_amd.mclbm\nexcept ImportError as e:\n"
            "    print('raised:', e); sys.exit(0)\nsys.exit(1)")
    p = subprocess.run([sys.executable, "-c", code, str(tmp_path)], capture_output=True, text=True, timeout=300)
    assert p.returncode == 0 and "no fallback" in p.stdout, (p.stdout, p.stderr[-1000:])


def test_plan_reports_alignment_and_validates_options(M):
    p = M.make_params(40, 30, mu=0.05, nu=0.3, tau=0.55)
    assert M.mclbm_plan_align(p) == 256
    base, _ = M.mclbm_plan(p)
    for field, value in (("extrap", 2), ("extrap", -1), ("corner", 3), ("corner", -1), ("boundary_order", 3),
                         ("boundary_order", -1), ("time_levels", 2), ("diag_every", -1), ("reserved_", 1)):
        q = M.make_params(40, 30, mu=0.05, nu=0.3, tau=0.55)
        setattr(q, field, value)
        with pytest.raises(M.MclbmError) as e:
            M.mclbm_plan(q)
        assert e.value.code == M.MCLBM_EINVAL, (field, value)
    # the options of the fused step keep the arena; the multi-pass step holds
    # T and sigma in FP64 (48 B per node), the printed order two levels of them
    for kw in (dict(extrap=1), dict(corner=2), dict(diag_every=10)):
        assert M.mclbm_plan(M.make_params(40, 30, mu=0.05, nu=0.3, tau=0.55, **kw))[0] == base
    plane = 30 * 64
    b2, _ = M.mclbm_plan(M.make_params(40, 30, mu=0.05, nu=0.3, tau=0.55, boundary_order=2))
    bl, _ = M.mclbm_plan(M.make_params(40, 30, mu=0.05, nu=0.3, tau=0.55, time_levels=1))
    assert b2 >= base + 48 * plane and bl >= base + 96 * plane
    # zero means first order, for a zero-initialised struct
    q = M.make_params(40, 30, mu=0.05, nu=0.3, tau=0.55)
    q.boundary_order = 0
    assert M.mclbm_plan(q)[0] == base


def test_table_program_validation_without_gpu(M):
    p = M.make_params(16, 16, mu=0.05, nu=0.3, tau=1.0)
    nbytes, _ = M.mclbm_plan(p)
    h = M.mclbm_create(p, 1 << 20, nbytes, 0)
    try:
        spec = M.make_side("neumann", "table", (1e-3, 0.0))  # no table
        with pytest.raises(M.MclbmError) as e:
            M.mclbm_set_side(h, 1, spec)
        assert e.value.code == M.MCLBM_EINVAL
        with pytest.raises(M.MclbmError) as e:
            M.mclbm_set_side(h, 1, M.make_side("neumann", "table", (1e-3, 0.0), table=[0.0, float("nan")]))
        assert e.value.code == M.MCLBM_EINVAL
        spec = M.make_side("neumann", "table", (1e-3, 0.0), table=[0.0, 0.5, 1.0])
        M.mclbm_set_side(h, 1, spec)
    finally:
        M.mclbm_destroy(h)


def _header(nx, ny, precision, material, time_levels, step, f_bytes, u_bytes, extra, magic=b"MCLBMCK1", version=2):
    import struct
    return struct.pack("<8s6iq3Q", magic, version, nx, ny, precision, material, time_levels, step,
                       f_bytes, u_bytes, extra)


def test_checkpoint_header_is_checked_without_gpu(M):
    """mclbm_load rejects a short buffer, a foreign file and a checkpoint of
    another lattice, storage or time order with EINVAL, before any copy."""
    import numpy as np
    p = M.make_params(16, 16, mu=0.05, nu=0.3, tau=1.0, precision="f32")
    nbytes, _ = M.mclbm_plan(p)
    h = M.mclbm_create(p, 1 << 20, nbytes, 0)
    try:
        need = M.mclbm_state_bytes(h)
        plane = 16 * 64
        f_bytes, u_bytes = 36 * plane, 16 * plane
        assert need == 64 + f_bytes + u_bytes
        cases = [
            _header(16, 16, 1, 0, 0, 5, f_bytes, u_bytes, 0)[:40],                  # short
            _header(16, 16, 1, 0, 0, 5, f_bytes, u_bytes, 0, magic=b"NOTMCLBM"),    # foreign
            _header(16, 16, 1, 0, 0, 5, f_bytes, u_bytes, 0, version=1),            # the planar format
            _header(17, 16, 1, 0, 0, 5, f_bytes, u_bytes, 0),                       # lattice
            _header(16, 16, 0, 0, 0, 5, 72 * plane, u_bytes, 0),                    # storage
            _header(16, 16, 1, 1, 0, 5, f_bytes, u_bytes, 0),                       # material
            _header(16, 16, 1, 0, 1, 5, f_bytes, u_bytes, 48 * plane),              # time order
            _header(16, 16, 1, 0, 0, -3, f_bytes, u_bytes, 0),                      # step
        ]
        for k, hd in enumerate(cases):
            buf = np.zeros(max(len(hd), 64 if k else len(hd)) + (need if k else 0), dtype=np.uint8)
            buf[:len(hd)] = np.frombuffer(hd, dtype=np.uint8)
            n = len(hd) if k == 0 else buf.size
            with pytest.raises(M.MclbmError) as e:
                M.mclbm_load(h, buf.ctypes.data, n, 0)
            assert e.value.code == M.MCLBM_EINVAL, k
        # a matching header over a buffer shorter than the state
        hd = _header(16, 16, 1, 0, 0, 5, f_bytes, u_bytes, 0)
        buf = np.zeros(need, dtype=np.uint8)
        buf[:64] = np.frombuffer(hd, dtype=np.uint8)
        with pytest.raises(M.MclbmError) as e:
            M.mclbm_load(h, buf.ctypes.data, need - 1, 0)
        assert e.value.code == M.MCLBM_EINVAL
        # saving needs an initialised simulation and room for the state
        with pytest.raises(M.MclbmError) as e:
            M.mclbm_save(h, buf.ctypes.data, need, 0)
        assert e.value.code == M.MCLBM_ESTATE
    finally:
        M.mclbm_destroy(h)
