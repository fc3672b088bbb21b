"""Benchmark of the moment-chain LBM time step on one MI355X.

Workload: St. Venant-Kirchhoff uniaxial tension on an 8192 x 8192 D2Q9 lattice
(mu = 0.05, nu = 0.3, tau = 0.55; left edge held, right edge pulled at
3.2e-3 dx per step, top and bottom traction-free), synthetic and seeded.
A step is one launch of the fused step kernel over the whole lattice; inputs
are resident in HBM before timing starts.  The headline value is MLUPS with
FP32 population storage (FP64 displacement); the FP64 mode is reported beside
it.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode both|f32|f64]
                  [--n 8192] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, published
# algorithmic HBM bytes per lattice update: 9 populations read + written,
# u (2 x FP64) read + written
BYTES_PER_LUP = {"f32": 9 * 4 * 2 + 2 * 8 * 2, "f64": 9 * 8 * 2 + 2 * 8 * 2}
KERNEL_SRC = os.path.join(ROOT, "paper_2502_00920_amd", "csrc", "mclbm_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for name in ("mclbm_kernels.hip", "mclbm_device.hpp"):
        with open(os.path.join(ROOT, "paper_2502_00920_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(mode: str, nodes: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    rec = t.get(mode)
    if not rec or rec.get("nodes") != nodes:
        return None
    return rec.get("bytes_per_launch")


def time_mode(mode: str, n: int, steps: int, warmup: int):
    import torch
    from paper_2502_00920_amd import mclbm
    from paper_2502_00920_amd import workloads as W

    w = W.tension_large(n, steps=max(1000, steps + warmup))
    sim = mclbm.sim_from_workload(w, precision=mode)
    sim.init()  # u0 = 0: the run starts at rest, the right wall moves
    sim.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(sim.stream)
    sim.step(steps)
    stop.record(sim.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    d = sim.diag()
    nodes = n * n
    ms_step = ms / steps
    mlups = nodes * steps / (ms * 1e-3) / 1e6
    achieved = BYTES_PER_LUP[mode] * nodes / (ms_step * 1e-3) / 1e9
    traffic = measured_traffic(mode, nodes)
    res = {
        "value": mlups, "ms_per_step": ms_step,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "bytes_per_lup": BYTES_PER_LUP[mode]},
        "finite": not d["nonfinite"], "max_u": d["max_u"],
    }
    u = sim.read("u", host=False)
    del sim
    torch.cuda.empty_cache()
    return res, u


def copy_ceiling_gbs(nbytes: int = 4 << 30) -> float:
    """Bandwidth of a plain elementwise copy (read + write) of nbytes."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    a.record()
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)
    b.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return gbs


def cpu_baseline(target_s: float = 15.0):
    """The FP64 CPU oracle on the host cores: 1024 x 1024 subrun of the same
    workload, as many steps as fit in about target_s seconds."""
    import numpy as np  # noqa: F401
    import oracle
    from paper_2502_00920_amd import workloads as W

    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        threads = min(threads or 1, int(os.environ["OMP_NUM_THREADS"]))
    threads = max(1, min(int(threads or 1), 64))
    w = W.tension_large(1024, 1000)
    o = oracle.Oracle(w.nx, w.ny, mu=w.mu, nu=w.nu, tau=w.tau, material=w.material, threads=threads)
    for side, sd in w.sides.items():
        o.set_side(side, sd.bc, sd.kind, sd.amp, sd.t0, sd.t1, sd.width)
    o.init()
    t0 = time.perf_counter()
    o.step(2)
    per = (time.perf_counter() - t0) / 2
    k = max(2, min(1000, int(target_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    o.step(k)
    dt = time.perf_counter() - t0
    return {"value": w.nodes * k / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle, 1024x1024 SVK tension, {k} steps, {dt:.1f} s, "
                      f"{threads} OpenMP threads on {platform.processor() or platform.machine()}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--mode", choices=["both", "f32", "f64"], default="both")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the time step of one "
              "lattice runs on a single MI355X; see DESIGN.md for how it would shard)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)

    modes = ["f32", "f64"] if args.mode == "both" else [args.mode]
    results, fields = {}, {}
    for m in modes:
        results[m], fields[m] = time_mode(m, args.n, args.steps, args.warmup)
        print(f"# {m}: {results[m]['value']:.0f} MLUPS, {results[m]['ms_per_step']:.3f} ms/step, "
              f"{results[m]['roofline']['achieved']:.0f} GB/s", file=sys.stderr, flush=True)
    agree = None
    if "f32" in fields and "f64" in fields:
        a, b = fields["f32"], fields["f64"]
        agree = float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    del fields
    torch.cuda.empty_cache()
    copy = copy_ceiling_gbs()
    head = modes[0]
    r = results[head]
    line = {
        "metric": "MLUPS and HBM GB/s per step (FP32/mixed vs FP64); batched p50/p99 latency",
        "value": r["value"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": head, "data": "synthetic",
        "config": {"workload": f"tension{args.n}: St. Venant-Kirchhoff uniaxial tension, D2Q9 "
                               f"{args.n}x{args.n}, mu=0.05, nu=0.3, tau=0.55, left held, right "
                               "pulled 3.2e-3 dx/step, top/bottom traction-free",
                   "storage": "populations " + head + ", displacement f64"},
        "hbm_gbs": r["roofline"]["achieved"],
        "roofline": {k: v for k, v in r["roofline"].items() if k != "bytes_per_lup"},
        "copy_ceiling_gbs": copy,
        "finite": r["finite"],
    }
    for m in modes[1:]:
        line[m] = {"value": results[m]["value"], "ms_per_step": results[m]["ms_per_step"],
                   "hbm_gbs": results[m]["roofline"]["achieved"],
                   "roofline": {k: v for k, v in results[m]["roofline"].items() if k != "bytes_per_lup"},
                   "finite": results[m]["finite"]}
    if agree is not None:
        line["f32_vs_f64_rel_l2_u"] = agree
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
