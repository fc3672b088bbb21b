"""The C ABI on its own: the stand-alone C++ program mclbm_demo (no Python,
no torch; it allocates its arena and stream with HIP itself) runs a small
Dirichlet-pulled lattice, and its displacement matches the oracle's."""
import os
import subprocess

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEMO = os.path.join(ROOT, "paper_2502_00920_amd", "mclbm_demo")
TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_c_abi_demo_against_oracle(tmp_path, precision):
    print(f"\n[case] C ABI demo {precision}", flush=True)
    assert os.path.exists(DEMO), f"{DEMO} is missing: build with python -m paper_2502_00920_amd.build"
    out = tmp_path / f"u_{precision}.bin"
    r = subprocess.run([DEMO, str(out), precision, "300"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    print(r.stdout.strip(), flush=True)
    u = np.fromfile(out, dtype=np.float64).reshape(2, 45, 70)
    o = oracle.Oracle(70, 45, mu=0.05, nu=0.2, tau=0.55, material="svk", threads=min(8, os.cpu_count() or 1))
    o.set_side("left", "dirichlet")
    o.set_side("right", "dirichlet", "disp_ramp", (0.5, 0.0), 0, 200)
    o.set_side("bottom", "neumann")
    o.set_side("top", "neumann")
    o.init()
    o.step(300)
    ref = o.read("u")
    e = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    print(f"rel L2 u {e:.2e}", flush=True)
    assert e <= TOL[precision]
