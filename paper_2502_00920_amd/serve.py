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
prints one JSON line: the stream batched with FP32, FP64 and FP16 population
storage, all requests queued at once (updates run per second, updates of the
requests that finished stably per second, requests per second, and the
unstable requests, beyond the CFL bound nu > 1/4 and within it); open-loop
p50/p99 latency with Poisson arrivals at the given fraction of the FP32 request
rate; one-at-a-time plain FP64 solves of a sample spread evenly over the
stream's work per request (checked every 500 steps, so that diverging runs stop
early as in the server); the gains of batching (batched FP64 over one at a
time) and of FP32 storage; and each batched format's error against the
one-at-a-time FP64 results on the sample's stable requests.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
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
    ran), and in updates of the requests that finished stably per second."""
    import torch
    from . import mclbm
    sv = mclbm.Server(precision=precision, **server_kw)
    t0 = time.perf_counter()
    ids = [_submit(sv, r) for r in reqs]
    sv.drain()
    dt = time.perf_counter() - t0
    res = {i: sv.result(rid) for i, rid in enumerate(ids)}
    ran = sum(r["nx"] * r["ny"] * sv.steps(rid) for r, rid in zip(reqs, ids))
    stable = sum(r["nx"] * r["ny"] * r["nsteps"] for i, r in enumerate(reqs) if res[i][1] == 0)
    del sv
    torch.cuda.empty_cache()
    return {"capacity_lups_per_s": ran / dt, "completed_lups_per_s": stable / dt, "closed_loop_seconds": dt,
            "requests_per_s": len(reqs) / dt, **unstable_counts(reqs, {i: v[1] for i, v in res.items()})}, res


def unstable_counts(reqs, status):
    """Requests that lost stability (status != 0), beyond the CFL bound of
    first-order boundary stencils (nu > 1/4, Sect. 3.2) and within it."""
    bad = [r for r in reqs if status[r["id"]] != 0]
    return {"unstable": len(bad), "unstable_nu_above_quarter": sum(1 for r in bad if r["nu"] > 0.25),
            "unstable_nu_within_quarter": sum(1 for r in bad if r["nu"] <= 0.25),
            "requests_nu_above_quarter": sum(1 for r in reqs if r["nu"] > 0.25)}


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


def run_sequential(reqs, precision="f64", check_every=500):
    """One simulation at a time with the plain single-lattice path, checked for
    values that are not finite every check_every steps (as the server scans
    after each round), so that a diverging run stops early there too."""
    import torch
    from . import mclbm
    out, status, ran = {}, {}, 0.0
    t0 = time.perf_counter()
    for r in reqs:
        s = mclbm.Sim(r["nx"], r["ny"], mu=r["mu"], nu=r["nu"], tau=r["tau"], material=r["material"],
                      precision=precision)
        for name, spec in r["sides"].items():
            args = (spec,) if isinstance(spec, str) else tuple(spec)
            s.set_side(name, *args)
        s.init()
        ok, n = s.step_checked(r["nsteps"], every=check_every)
        ran += r["nx"] * r["ny"] * n
        status[r["id"]] = 0 if ok else mclbm.MCLBM_EUNSTABLE
        out[r["id"]] = s.read("u")
        del s
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    torch.cuda.empty_cache()
    stable = sum(r["nx"] * r["ny"] * r["nsteps"] for r in reqs if status[r["id"]] == 0)
    return {"lups_per_s": ran / dt, "completed_lups_per_s": stable / dt, "requests": len(reqs), "seconds": dt,
            **unstable_counts(reqs, status)}, out, status


def stratified(reqs, k):
    """k requests spread evenly over the stream's range of work (updates per
    request), the middle of each of k equal-count bins."""
    order = sorted(reqs, key=lambda r: r["nx"] * r["ny"] * r["nsteps"])
    k = min(k, len(order))
    return [order[int((i + 0.5) * len(order) / k)] for i in range(k)]


def _phase(name, t0):
    print(f"[serve] {name} done at {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)


def serving_report(n=1000, seed=0, steps=(1000, 20000), load=0.8, baseline=40, **server_kw):
    t0 = time.perf_counter()
    reqs = make_requests(n, seed=seed, steps=steps)
    f32, res = run_closed(reqs, **server_kw)
    _phase("batched FP32", t0)
    # Poisson arrivals at `load` times the closed loop's request rate
    opn = run_open(reqs, rate=load * len(reqs) / f32["closed_loop_seconds"], **server_kw)
    _phase("open loop FP32", t0)
    # the same stream batched with FP64 (the batching gain alone) and 16-bit storage
    f64, res64 = run_closed(reqs, precision="f64", **server_kw)
    _phase("batched FP64", t0)
    f16, res16 = run_closed(reqs, precision="f16", **server_kw)
    _phase("batched FP16", t0)
    # one-at-a-time plain FP64 on a sample spread over the stream's sizes and lengths
    sub = stratified(reqs, baseline)
    seq, useq, sseq = run_sequential(sub, "f64")
    _phase("one-at-a-time FP64", t0)
    sample_ids = {r["id"] for r in sub}

    def max_err(batched):
        # accuracy of batched results against the one-at-a-time FP64 ones, on the
        # sample's requests that both finished stably
        errs = []
        for r in sub:
            st, status, u = batched[r["id"]]
            ref = useq[r["id"]]
            if status == 0 and sseq[r["id"]] == 0 and np.linalg.norm(ref) > 0:
                errs.append(float(np.linalg.norm(u - ref) / np.linalg.norm(ref)))
        return {"max": max(errs) if errs else None, "compared": len(errs)}

    agree64 = sum(1 for i in sample_ids if (res64[i][1] == 0) == (sseq[i] == 0))
    return {"workload": f"{n} requests, sides 64..1024, SVK/NH, nu 0..0.45, tension/shear/cantilever, "
                        f"{steps[0]}..{steps[1]} steps, seed {seed}",
            "batched_f32": f32,
            "open_loop_f32": opn,
            "batched_f64": f64,
            "batched_f16": f16,
            "sequential_f64": {**seq, "sample": f"{len(sub)} requests at evenly spaced quantiles of the "
                                                "stream's updates per request",
                               "stable_verdict_agrees_with_batched_f64": f"{agree64} of {len(sub)}"},
            "speedup_vs_sequential_f64": f32["capacity_lups_per_s"] / seq["lups_per_s"],
            "speedup_completed_vs_sequential_f64": f32["completed_lups_per_s"] / seq["completed_lups_per_s"]
            if seq["completed_lups_per_s"] > 0 else None,
            "batching_gain_f64": f64["capacity_lups_per_s"] / seq["lups_per_s"],
            "storage_gain_f32_over_f64_batched": f32["capacity_lups_per_s"] / f64["capacity_lups_per_s"],
            "batched_f32_vs_sequential_f64_rel_l2_u": max_err(res),
            "batched_f64_vs_sequential_f64_rel_l2_u": max_err(res64),
            "batched_f16_vs_sequential_f64_rel_l2_u": max_err(res16)}


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
