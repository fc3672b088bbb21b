"""Serving workload and drivers for the continuous-batching server (mclbm.Server).

The request stream: square lattices with sides log-uniform in [64, 1024];
St. Venant-Kirchhoff or neo-Hooke with equal odds; nu uniform in [0, 0.45];
mu = 0.05, tau = 0.55; step counts uniform in [1000, 20000]; one of three load
cases, each on the walls of the paper's experiments (Sect. 4), with loads that
scale with the lattice but move no wall faster than a slow pull:
  tension     left held, right pulled at constant speed over the first two
              thirds of the steps, then held; it moves by 5 % of the side (a 5 %
              stretch) or, if that needs more, by 3.2e-3 dX per step
  shear       bottom held, top moved sideways over the first half of the steps,
              then held; by 5 % of the side (shear 0.05) or at most 6.4e-3 dX per
              step; left and right free
  cantilever  left held, transverse Gaussian traction pulse on the right (peak
              1e-3 mu, width 200 steps, centred at step 800, free after 1600)
Arrivals are Poisson.  Runs with nu above 1/4 break the CFL bound of first-order
boundary stencils (Sect. 3.2) and most of them diverge, as do some long runs at
nu near 0; they are reported as unstable and left out of the latency figures.

  python -m paper_2502_00920_amd.serve [--requests 1000] [--seed 0]
      [--steps-min 1000] [--steps-max 20000] [--load 0.8] [--baseline 40]
prints one JSON line: batched capacity (lattice updates run per second, and
requests per second), open-loop p50/p99 latency with Poisson arrivals at the
given fraction of that request rate, and the throughput of one-at-a-time FP64
solves.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np


def make_requests(n, seed=0, steps=(1000, 20000), sides=(64, 1024), mu=0.05, tau=0.55):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        side = int(round(math.exp(rng.uniform(math.log(sides[0]), math.log(sides[1])))))
        material = "svk" if rng.random() < 0.5 else "neohooke"
        nu = float(rng.uniform(0.0, 0.45))
        case = ("tension", "shear", "cantilever")[int(rng.integers(0, 3))]
        nsteps = int(rng.integers(steps[0], steps[1] + 1))
        if case == "tension":
            t1 = max(1, (2 * nsteps) // 3)
            d = min(0.05 * side, 3.2e-3 * t1)
            walls = {"left": ("dirichlet",), "right": ("dirichlet", "disp_ramp", (d, 0.0), 0, t1),
                     "bottom": "neumann", "top": "neumann"}
        elif case == "shear":
            t1 = max(1, nsteps // 2)
            d = min(0.05 * side, 6.4e-3 * t1)
            walls = {"bottom": ("dirichlet",), "top": ("dirichlet", "disp_ramp", (d, 0.0), 0, t1),
                     "left": "neumann", "right": "neumann"}
        else:
            walls = {"left": ("dirichlet",), "right": ("neumann", "gauss", (0.0, 1e-3 * mu), 800, 1600, 200),
                     "bottom": "neumann", "top": "neumann"}
        out.append(dict(id=i, nx=side, ny=side, mu=mu, nu=nu, tau=tau, material=material, sides=walls,
                        nsteps=nsteps, case=case))
    return out


def lups(reqs):
    return float(sum(r["nx"] * r["ny"] * r["nsteps"] for r in reqs))


def _submit(server, r):
    return server.submit(r["nx"], r["ny"], mu=r["mu"], nu=r["nu"], tau=r["tau"], material=r["material"],
                         sides=r["sides"], nsteps=r["nsteps"])


def run_closed(reqs, precision="f32", **server_kw):
    """Every request queued at once: the server's capacity in lattice updates
    run per second (unstable requests stop early and count only the steps they
    ran)."""
    import torch
    from . import mclbm
    sv = mclbm.Server(precision=precision, **server_kw)
    t0 = time.perf_counter()
    ids = [_submit(sv, r) for r in reqs]
    sv.drain()
    dt = time.perf_counter() - t0
    res = {i: sv.result(rid) for i, rid in enumerate(ids)}
    ran = sum(r["nx"] * r["ny"] * sv.steps(rid) for r, rid in zip(reqs, ids))
    del sv
    torch.cuda.empty_cache()
    return ran / dt, dt, res


def run_open(reqs, rate, seed=1, precision="f32", **server_kw):
    """Poisson arrivals at `rate` requests per second; latency = completion - arrival."""
    import torch
    from . import mclbm
    rng = np.random.default_rng(seed)
    arrival = np.cumsum(rng.exponential(1.0 / rate, size=len(reqs)))
    sv = mclbm.Server(precision=precision, **server_kw)
    t0 = time.perf_counter()
    nxt, rid_of, done_at = 0, {}, {}
    while len(done_at) < len(reqs):
        now = time.perf_counter() - t0
        while nxt < len(reqs) and arrival[nxt] <= now:
            rid_of[_submit(sv, reqs[nxt])] = nxt
            nxt += 1
        for rid in sv.progress():
            done_at[rid_of[rid]] = time.perf_counter() - t0
        w, a, _ = sv.counts()
        if w == 0 and a == 0 and nxt < len(reqs):
            time.sleep(max(0.0, min(arrival[nxt] - (time.perf_counter() - t0), 0.05)))
    total = time.perf_counter() - t0
    status = {i: sv.result(rid)[1] for rid, i in rid_of.items()}
    ran = sum(reqs[i]["nx"] * reqs[i]["ny"] * sv.steps(rid) for rid, i in rid_of.items())
    del sv
    torch.cuda.empty_cache()
    lat = np.array([done_at[i] - arrival[i] for i in range(len(reqs)) if status[i] == 0])
    return {"requests": len(reqs), "rate_per_s": rate, "seconds": total,
            "lups_per_s": ran / total, "unstable": int(sum(1 for s in status.values() if s != 0)),
            "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_s": float(np.percentile(lat, 99)) if lat.size else None}


def run_sequential(reqs, precision="f64"):
    """One simulation at a time with the plain single-lattice path."""
    import torch
    from . import mclbm
    out = {}
    t0 = time.perf_counter()
    for r in reqs:
        s = mclbm.Sim(r["nx"], r["ny"], mu=r["mu"], nu=r["nu"], tau=r["tau"], material=r["material"],
                      precision=precision)
        for name, spec in r["sides"].items():
            args = (spec,) if isinstance(spec, str) else tuple(spec)
            s.set_side(name, *args)
        s.init()
        s.step(r["nsteps"])
        out[r["id"]] = s.read("u")
        del s
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    torch.cuda.empty_cache()
    return lups(reqs) / dt, dt, out


def serving_report(n=1000, seed=0, steps=(1000, 20000), load=0.8, baseline=40, **server_kw):
    reqs = make_requests(n, seed=seed, steps=steps)
    cap, cap_s, res = run_closed(reqs, **server_kw)
    # Poisson arrivals at `load` times the closed loop's request rate
    opn = run_open(reqs, rate=load * len(reqs) / cap_s, **server_kw)
    # the same stream with 16-bit population storage
    cap16, cap16_s, res16 = run_closed(reqs, precision="f16", **server_kw)
    sub = reqs[:baseline]
    seq, seq_s, useq = run_sequential(sub, "f64")

    def max_err(batched):
        # accuracy of batched results against the one-at-a-time FP64 ones
        errs = []
        for r in sub:
            st, status, u = batched[r["id"]]
            ref = useq[r["id"]]
            if status == 0 and np.all(np.isfinite(ref)) and np.linalg.norm(ref) > 0:
                errs.append(float(np.linalg.norm(u - ref) / np.linalg.norm(ref)))
        return max(errs) if errs else None

    return {"workload": f"{n} requests, sides 64..1024, SVK/NH, nu 0..0.45, tension/shear/cantilever, "
                        f"{steps[0]}..{steps[1]} steps, seed {seed}",
            "batched_f32": {"capacity_lups_per_s": cap, "closed_loop_seconds": cap_s,
                            "requests_per_s": len(reqs) / cap_s,
                            "unstable": int(sum(1 for v in res.values() if v[1] != 0))},
            "open_loop_f32": opn,
            "batched_f16": {"capacity_lups_per_s": cap16, "closed_loop_seconds": cap16_s,
                            "unstable": int(sum(1 for v in res16.values() if v[1] != 0))},
            "sequential_f64": {"lups_per_s": seq, "requests": len(sub), "seconds": seq_s},
            "speedup_vs_sequential_f64": cap / seq,
            "batched_f32_vs_sequential_f64_rel_l2_u_max": max_err(res),
            "batched_f16_vs_sequential_f64_rel_l2_u_max": max_err(res16)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=1000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--steps-min", type=int, default=1000)
    ap.add_argument("--steps-max", type=int, default=20000)
    ap.add_argument("--load", type=float, default=0.8)
    ap.add_argument("--baseline", type=int, default=40)
    a = ap.parse_args()
    print(json.dumps(serving_report(a.requests, a.seed, (a.steps_min, a.steps_max), a.load, a.baseline)),
          flush=True)


if __name__ == "__main__":
    main()
