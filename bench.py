"""Benchmark of the moment-chain LBM time step on one MI355X.

Workload: St. Venant-Kirchhoff uniaxial tension on an 8192 x 8192 D2Q9 lattice
(mu = 0.05, nu = 0.3, tau = 0.55; left edge held, right edge pulled at
3.2e-3 dx per step, top and bottom traction-free), synthetic and seeded.
A step is one launch of march_kernel over every node (its wall blocks update
the wall nodes in the same launch); inputs are resident in HBM before timing
starts.  The headline value is MLUPS with
FP32 population storage (FP64 displacement); FP64 and the 16-bit storage modes
(FP16, BF16) are reported beside it, each format's error against the FP64
oracle on the 1024 x 1024 subrun (from the CPU-baseline leg), and a shortened
run of the serving workload (batched throughput, p50/p99 latency).  The
roofline figures are those of march_kernel, timed with HIP events around each
of its launches in the timed region.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode all|f32|f64|f16|bf16]
                  [--n 8192] [--no-cpu-baseline] [--no-serving]
  python bench.py --ingest-counters FETCH_DIR WRITE_DIR   (no GPU: rocprofv3
                  counter files -> profiles/step_kernel_traffic.json)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, published
# algorithmic HBM bytes per lattice update, the method's state read and written
# once: 9 populations, u (2 x FP64) and j (2 values of the arithmetic type)
BYTES_PER_LUP = {"f32": 9 * 4 * 2 + 2 * 8 * 2 + 2 * 4 * 2, "f64": 9 * 8 * 2 + 2 * 8 * 2 + 2 * 8 * 2,
                 "f16": 9 * 2 * 2 + 2 * 8 * 2 + 2 * 4 * 2, "bf16": 9 * 2 * 2 + 2 * 8 * 2 + 2 * 4 * 2}
# what this kernel must move: it keeps no j (it is recovered from the stored
# post-collision populations), so 16 B (FP64: 32 B) less
COMPULSORY_BYTES_PER_LUP = {"f32": 9 * 4 * 2 + 2 * 8 * 2, "f64": 9 * 8 * 2 + 2 * 8 * 2,
                            "f16": 9 * 2 * 2 + 2 * 8 * 2, "bf16": 9 * 2 * 2 + 2 * 8 * 2}
KERNEL_SRC = os.path.join(ROOT, "paper_2502_00920_amd", "csrc", "mclbm_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")
COPY_BYTES = 2 << 30  # bytes read (and written) by one launch of the calibration copy


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
    # the timed region: steps steps on the simulation's stream, with HIP events
    # around each launch recorded by the library
    start.record(sim.stream)
    ms_steps, ms_kernel = sim.step_timed(steps)
    stop.record(sim.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    d = sim.diag()
    nodes = n * n
    ms_step = ms / steps
    mlups = nodes * steps / (ms * 1e-3) / 1e6
    # march_kernel updates every node once per launch: its own wall blocks, or
    # the wall kernel after it, the 4 n - 4 wall nodes
    alg_bytes = BYTES_PER_LUP[mode] * nodes
    comp_bytes = COMPULSORY_BYTES_PER_LUP[mode] * nodes
    achieved = alg_bytes / (ms_kernel * 1e-3) / 1e9
    traffic = measured_traffic(mode, nodes)
    res = {
        "value": mlups, "ms_per_step": ms_step, "step_gbs": alg_bytes / (ms_step * 1e-3) / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic},
        "roofline_compulsory": {"bytes_per_lup": COMPULSORY_BYTES_PER_LUP[mode],
                                "achieved": comp_bytes / (ms_kernel * 1e-3) / 1e9,
                                "frac": comp_bytes / (ms_kernel * 1e-3) / 1e9 / PEAK_HBM_GBS},
        "kernels": {"march_kernel_ms": ms_kernel, "step_ms_events": ms_steps,
                    "rest_of_step_ms": ms_steps - ms_kernel,
                    "algorithmic_bytes_per_launch": alg_bytes, "bytes_per_lup": BYTES_PER_LUP[mode],
                    "traffic_vs_algorithmic": None if traffic is None else traffic / alg_bytes,
                    "traffic_vs_compulsory": None if traffic is None else traffic / comp_bytes},
        "finite": not d["nonfinite"], "max_u": d["max_u"],
    }
    u = sim.read("u", host=False)
    del sim
    torch.cuda.empty_cache()
    return res, u


def copy_gbs(nbytes: int = COPY_BYTES) -> dict:
    """Copy bandwidth (read + write) over nbytes: the library's calibration copy
    (32-bit accesses, as the step kernel) and torch's vectorised elementwise copy."""
    import torch
    from paper_2502_00920_amd import mclbm
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    st = torch.cuda.current_stream()

    def timed(fn, reps=10):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        for _ in range(reps):
            fn()
        b.record(st)
        torch.cuda.synchronize()
        return 2 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9

    out = {"mclbm_copy": timed(lambda: mclbm.mclbm_copy(y.data_ptr(), x.data_ptr(), nbytes, st.cuda_stream)),
           "torch_elementwise": timed(lambda: torch.mul(x, 1.0, out=y))}
    del x, y
    torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo where there is one)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(n: int = 1024, steps: int = 1000):
    """The FP64 CPU oracle on the host's cores over the n x n subrun of the
    benchmark workload (all its steps).  Returns the baseline record and the
    oracle's final u and P, the reference for the per-format subrun errors."""
    import oracle
    from paper_2502_00920_amd import workloads as W

    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        threads = min(threads or 1, int(os.environ["OMP_NUM_THREADS"]))
    threads = max(1, min(int(threads or 1), 64))
    w = W.tension_large(n, steps)
    o = oracle.Oracle(w.nx, w.ny, mu=w.mu, nu=w.nu, tau=w.tau, material=w.material, threads=threads)
    for side, sd in w.sides.items():
        o.set_side(side, sd.bc, sd.kind, sd.amp, sd.t0, sd.t1, sd.width)
    o.init()
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    rec = {"value": w.nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"FP64 oracle, {n}x{n} subrun of the SVK tension workload, all {steps} steps, "
                     f"{dt:.1f} s, {threads} OpenMP threads on {cpu_model()}"}
    return rec, o.read("u"), o.read("p")


def subrun_errors(u_ref, p_ref, n: int = 1024, steps: int = 1000) -> dict:
    """Relative L2 error of u and P against the oracle's subrun, per storage format."""
    import numpy as np
    import torch
    from paper_2502_00920_amd import mclbm
    from paper_2502_00920_amd import workloads as W

    w = W.tension_large(n, steps)
    out = {"workload": f"tension{n}, {steps} steps (the subrun of the benchmark workload)"}
    for m in ("f64", "f32", "f16", "bf16"):
        sim = mclbm.sim_from_workload(w, precision=m)
        sim.init()
        sim.step(steps)
        u, pk = sim.read("u"), sim.read("p")
        out[m] = {"u": float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)),
                  "p": float(np.linalg.norm(pk - p_ref) / np.linalg.norm(p_ref))}
        del sim
        torch.cuda.empty_cache()
    return out


def serving(n: int = 200, steps=(1000, 4000), baseline: int = 20) -> dict:
    """A shortened run of the serving workload (the full one:
    python -m paper_2502_00920_amd.serve): batched FP32 capacity, open-loop
    p50/p99 latency at 0.8 of it, one-at-a-time FP64 throughput."""
    from paper_2502_00920_amd import serve
    return serve.serving_report(n=n, steps=steps, baseline=baseline)


def ingest_counters(fetch_dir: str, write_dir: str, n: int, out_path: str = TRAFFIC_FILE) -> dict:
    """Turn two rocprofv3 --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE;
    counter values in KiB per dispatch) into HBM bytes per launch of
    march_kernel, each counter scaled by what it reads for the library's copy
    kernel moving COPY_BYTES; writes out_path (the traffic file by default)."""
    import csv
    import glob

    def per_kernel(d, counter):
        vals = {}
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(path, newline="") as f:
                for row in csv.DictReader(f):
                    if row["Counter_Name"] != counter:
                        continue
                    name = row["Kernel_Name"]
                    # march_kernel<storage, material, ...>; the workload's material is
                    # St. Venant-Kirchhoff (0)
                    m = re.search(r"mclbm::march_kernel<(\d), 0\b", name)
                    key = (("f64", "f32", "f16", "bf16")[int(m.group(1))] if m else
                           "copy" if "mclbm::copy_kernel" in name else None)
                    if key:
                        vals.setdefault(key, []).append(float(row["Counter_Value"]) * 1024.0)
        return {k: sum(v) / len(v) for k, v in vals.items()}

    fetch, write = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    if "copy" not in fetch or "copy" not in write:
        raise SystemExit("no copy_kernel dispatch in the counter files: cannot calibrate")
    ff, fw = COPY_BYTES / fetch["copy"], COPY_BYTES / write["copy"]
    out = {"kernel_hash": kernel_hash(), "workload": f"tension{n}", "copy_bytes": COPY_BYTES,
           "fetch_factor": ff, "write_factor": fw}
    for m in ("f32", "f64", "f16", "bf16"):
        if m in fetch and m in write:
            rd, wr = fetch[m] * ff, write[m] * fw
            alg = BYTES_PER_LUP[m] * n * n
            comp = COMPULSORY_BYTES_PER_LUP[m] * n * n
            out[m] = {"nodes": n * n, "fetch_size_bytes": fetch[m], "write_size_bytes": write[m],
                      "read_bytes": rd, "written_bytes": wr, "bytes_per_launch": rd + wr,
                      "algorithmic_bytes": alg, "ratio": (rd + wr) / alg,
                      "compulsory_bytes": comp, "ratio_compulsory": (rd + wr) / comp}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    return out


def config_table() -> dict:
    """Per-configuration step rates: the GPU (MLUPS over a timed run of each
    storage mode; the small lattices are cache-resident, so these are effective
    rates, not roofline figures) and the CPU oracle on this host at one thread and
    at all of them (the CPU-baseline leg, on short samples of each)."""
    import torch
    import oracle
    from paper_2502_00920_amd import mclbm
    from paper_2502_00920_amd import workloads as W

    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cfgs = [(W.tension32(), ("f64", "f32"), 3000, 300),
            (W.shear128(0.25), ("f64", "f32"), 2000, 200),
            (W.beam2048(), ("f64", "f32", "f16"), 2000, 100),
            (W.tension_large(1024, 1000), ("f64", "f32", "f16"), 1000, 100)]
    out = {"host_threads": threads, "cpu": cpu_model(), "rows": []}
    for w, modes, gsteps, osteps in cfgs:
        row = {"workload": w.name, "nodes": w.nx * w.ny}
        for m in modes:
            s = mclbm.sim_from_workload(w, precision=m)
            s.init()
            s.step(10)
            torch.cuda.synchronize()
            ms, _ = s.step_timed(gsteps)
            row[f"gpu_{m}_mlups"] = w.nx * w.ny / ms / 1e3
            # the same steps launched back to back, events around the whole run
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            s.step(gsteps)
            e1.record()
            e1.synchronize()
            row[f"gpu_{m}_async_mlups"] = w.nx * w.ny * gsteps / e0.elapsed_time(e1) / 1e3
            del s
        torch.cuda.empty_cache()
        for t in (1, threads):
            o = oracle.Oracle(w.nx, w.ny, mu=w.mu, nu=w.nu, tau=w.tau, material=w.material, threads=t)
            for side, sd in w.sides.items():
                o.set_side(side, sd.bc, sd.kind, sd.amp, sd.t0, sd.t1, sd.width)
            o.init()
            t0 = time.perf_counter()
            o.step(osteps)
            row[f"oracle_{t}t_mlups"] = w.nx * w.ny * osteps / (time.perf_counter() - t0) / 1e6
        print("# " + json.dumps(row), file=sys.stderr, flush=True)
        out["rows"].append(row)
    return out


def error_growth(steps: int = 20000, every: int = 2000) -> dict:
    """Long-run error of each storage format against FP64 storage on the
    cantilever workload (2048x128 neo-Hooke, Gaussian traction pulse): the
    relative L2 of u every `every` steps, all modes advanced in lockstep on the
    GPU (the oracle would take hours for this run)."""
    import numpy as np
    import torch
    from paper_2502_00920_amd import mclbm
    from paper_2502_00920_amd import workloads as W

    w = W.beam2048()
    sims = {m: mclbm.sim_from_workload(w, precision=m) for m in ("f64", "f32", "f16", "bf16")}
    for s in sims.values():
        s.init()
    hist = []
    for n in range(every, steps + 1, every):
        for s in sims.values():
            s.step(every)
        ref = sims["f64"].read("u")
        row = {"step": n, "max_u_f64": float(np.abs(ref).max())}
        for m in ("f32", "f16", "bf16"):
            u = sims[m].read("u")
            row[m] = float(np.linalg.norm(u - ref) / max(np.linalg.norm(ref), 1e-300))
        print("# " + json.dumps(row), file=sys.stderr, flush=True)
        hist.append(row)
    del sims
    torch.cuda.empty_cache()
    return {"workload": f"{w.name}, FP64 storage as the reference", "history": hist}


def stability(precision: str = "f64", opts=None) -> dict:
    """The workloads at their full lengths: where each loses stability, and how
    fast a perturbation grows before that.  Each runs twice on the GPU, from its
    start and from its start plus seeded noise of 1e-12 dx on u; every `every`
    steps the largest |u| and the relative L2 distance of the two runs' u are
    recorded, until the run is no longer finite or its steps are done.  The
    growth rate is the slope of ln(distance) per step over the checkpoints where
    the distance lies between 1e-9 and 1e-3 (the perturbation still small).
    Where the two runs differ most at the last finite checkpoint is recorded
    (node and distance from the nearest wall).  opts: options of the step
    (mclbm.Sim keywords: extrap, corner, tau_plus, boundary_order, time_levels)."""
    import math
    import numpy as np
    import torch
    from paper_2502_00920_amd import mclbm
    from paper_2502_00920_amd import workloads as W

    cases = [(W.tension32(), 50), (W.shear128(0.0), 100), (W.shear128(0.25), 100), (W.shear128(0.45), 5),
             (W.beam2048(), 500)]
    opts = dict(opts or {})
    out = {"precision": precision, "options": opts, "perturbation": "uniform noise of 1e-12 dx on u0, seed 99",
           "rows": []}
    for w, every in cases:
        a, b = mclbm.sim_from_workload(w, precision, **opts), mclbm.sim_from_workload(w, precision, **opts)
        u0 = w.u0()
        a.init(u0)
        b.init(u0 + W.random_field(w.nx, w.ny, 1e-12 * w.dx, 99))
        hist, diverged, where = [], None, None
        for n in range(every, w.steps + 1, every):
            a.step(every)
            b.step(every)
            ua, ub = a.read("u"), b.read("u")
            umax = float(np.abs(ua).max()) if np.isfinite(ua).all() else float("inf")
            d = float(np.linalg.norm(ua - ub) / max(np.linalg.norm(ua), 1e-300)) if math.isfinite(umax) else float("inf")
            hist.append((n, umax, d))
            if not math.isfinite(umax) or umax > 1e3 * w.nx * w.dx:
                diverged = n
                break
            diff = np.abs(ua - ub).max(axis=0)
            y, x = np.unravel_index(int(np.argmax(diff)), diff.shape)
            where = {"step": n, "node": [int(x), int(y)],
                     "from_wall": int(min(x, w.nx - 1 - x, y, w.ny - 1 - y))}
        pts = [(n, math.log(d)) for n, _, d in hist if 1e-9 < d < 1e-3]
        rate = None
        if len(pts) >= 3:
            xs, ys = np.array([p[0] for p in pts], float), np.array([p[1] for p in pts])
            rate = float(np.polyfit(xs, ys, 1)[0])
        row = {"workload": w.name, "nu": w.nu, "tau": w.tau, "steps": w.steps, "diverged_by": diverged,
               "largest_difference_before": where,
               "growth_rate_per_step": rate,
               "growth_factor_per_step": None if rate is None else math.exp(rate),
               "history": [(n, round(u, 6), float(f"{d:.3e}")) for n, u, d in hist[:: max(1, len(hist) // 40)]]}
        print("# " + json.dumps({k: v for k, v in row.items() if k != "history"}), file=sys.stderr, flush=True)
        out["rows"].append(row)
        del a, b
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--mode", choices=["all", "f32", "f64", "f16", "bf16"], default="all")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--error-growth", action="store_true",
                    help="print the long-run error of each storage format against FP64 as one JSON line and exit")
    ap.add_argument("--stability", choices=["f64", "f32"],
                    help="run the workloads at their full lengths twice (perturbed start) and print where each "
                         "loses stability and how fast perturbations grow, as one JSON line, and exit")
    ap.add_argument("--stability-opts", default="{}",
                    help="with --stability: step options as JSON, e.g. '{\"tau_plus\": 1.0}'")
    ap.add_argument("--configs", action="store_true",
                    help="print the per-configuration rates (GPU and CPU oracle) as one JSON line and exit")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the traffic file from two rocprofv3 --pmc runs of this script and exit")
    args = ap.parse_args()
    if args.ingest_counters:
        print(json.dumps(ingest_counters(*args.ingest_counters, args.n), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the time step of one "
              "lattice runs on a single MI355X; across GPUs the lattice would split into slabs along y "
              "with one halo exchange per step)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)

    if args.configs:
        print(json.dumps(config_table()), flush=True)
        return
    if args.error_growth:
        print(json.dumps(error_growth()), flush=True)
        return
    if args.stability:
        print(json.dumps(stability(args.stability, json.loads(args.stability_opts))), flush=True)
        return

    modes = ["f32", "f64", "f16", "bf16"] if args.mode == "all" else [args.mode]
    results, fields = {}, {}
    for m in modes:
        results[m], fields[m] = time_mode(m, args.n, args.steps, args.warmup)
        print(f"# {m}: {results[m]['value']:.0f} MLUPS, {results[m]['ms_per_step']:.3f} ms/step, "
              f"step {results[m]['step_gbs']:.0f} GB/s, march_kernel "
              f"{results[m]['roofline']['achieved']:.0f} GB/s", file=sys.stderr, flush=True)
    agree = None
    if "f64" in fields:
        b = fields["f64"]
        agree = {m: float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) for m, a in fields.items() if m != "f64"}
    del fields
    torch.cuda.empty_cache()
    copy = copy_gbs()
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
                   "storage": "populations " + head + "; displacement, moments, collision and wall rules f64"},
        "hbm_gbs": r["step_gbs"],
        "roofline": r["roofline"],
        "kernels": r["kernels"],
        "copy_gbs": copy,
        "finite": r["finite"],
    }
    for m in modes[1:]:
        line[m] = {"value": results[m]["value"], "ms_per_step": results[m]["ms_per_step"],
                   "hbm_gbs": results[m]["step_gbs"],
                   "roofline": results[m]["roofline"], "kernels": results[m]["kernels"],
                   "finite": results[m]["finite"]}
    if agree:
        line["rel_l2_u_vs_f64_same_run"] = agree
    if not args.no_serving:
        line["serving"] = serving()
    if not args.no_cpu_baseline:
        line["cpu_baseline"], u_ref, p_ref = cpu_baseline()
        line["subrun_error_vs_fp64_oracle"] = subrun_errors(u_ref, p_ref)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
