"""Writes beam2048_fp_order_drift.json: how far two FP64 builds of the oracle
that differ only in the rounding order of their arithmetic drift apart on the
cantilever workload (2048 x 128 neo-Hooke, Gaussian traction pulse).

One build is the oracle's own (-O2 -ffp-contract=off); the other fuses
multiplies and adds (-O2 -mfma -ffp-contract=fast), as a GPU compiler does.
Both run the same steps from the same start; the relative L2 difference of u
and P between them is recorded at the checkpoints.  This is the scale at which
two correct FP64 implementations of the step disagree on this workload, the
reference for the long-horizon parity bar of the GPU tests.

Usage: python tests/golden/make_fp_order_drift.py [steps ...]   (about 2 minutes
on 8 threads for the default checkpoints 1000, 2000, 3000, 4000)
"""
import json
import os
import subprocess
import sys
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "beam2048_fp_order_drift.json")

CHILD = r"""
import sys, numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
from paper_2502_00920_amd import workloads as W
w = W.beam2048()
o = oracle.Oracle(w.nx, w.ny, mu=w.mu, nu=w.nu, tau=w.tau, material=w.material, threads=int(sys.argv[3]))
for side, sd in w.sides.items():
    o.set_side(side, sd.bc, sd.kind, sd.amp, sd.t0, sd.t1, sd.width)
o.init(w.u0())
for k, n in enumerate(int(a) for a in sys.argv[4:]):
    o.step(n - o.n)
    np.save(f"{sys.argv[2]}_u{k}.npy", o.read("u"))
    np.save(f"{sys.argv[2]}_p{k}.npy", o.read("p"))
    print(n, flush=True)
"""


def main():
    stops = [int(a) for a in sys.argv[1:]] or [1000, 2000, 3000, 4000]
    threads = str(min(16, os.cpu_count() or 1))
    src = os.path.join(ROOT, "oracle", "mclbm_oracle.c")
    builds = {"contract_off": ["-O2", "-ffp-contract=off", "-fno-fast-math"],
              "fma": ["-O2", "-mfma", "-ffp-contract=fast", "-fno-fast-math"]}
    with tempfile.TemporaryDirectory() as d:
        for name, flags in builds.items():
            lib = os.path.join(d, f"liboracle_{name}.so")
            subprocess.check_call(["gcc", *flags, "-fopenmp", "-fPIC", "-shared", "-o", lib, src, "-lm"])
            env = dict(os.environ, MCLBM_ORACLE_LIB=lib)
            subprocess.check_call([sys.executable, "-c", CHILD, ROOT, os.path.join(d, name), threads,
                                   *map(str, stops)], env=env)
        rec = {"workload": "beam2048x128 (neo-Hooke cantilever, Gaussian traction pulse), FP64 oracle",
               "builds": {k: " ".join(v) for k, v in builds.items()}, "rows": []}
        for k, n in enumerate(stops):
            row = {"step": n}
            for f in ("u", "p"):
                a = np.load(os.path.join(d, f"contract_off_{f}{k}.npy"))
                b = np.load(os.path.join(d, f"fma_{f}{k}.npy"))
                row[f] = float(np.linalg.norm(a - b) / np.linalg.norm(a))
            rec["rows"].append(row)
            print(row, flush=True)
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
