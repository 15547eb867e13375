#!/usr/bin/env python3
"""Local approximate GP prediction throughput on one MI355X.

One step = the whole hot path over the predictive set of the uniform 8-d
workload (N = 1e6 design points, M = 1e4 locations, n = 50, 1000 nearest
candidates, exhaustive greedy ALC search): candidate kNN, then the local
design search, partitioned-inverse updates and prediction.  Inputs are
resident in HBM before timing starts.  The ray-search form (10 rays) runs on
the same inputs and is reported beside it, as is the CPU oracle on a bounded
sample of locations.

    python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 (matrix and vector)
HBM_PEAK_GBS = 8000.0


def scoring_flops(n0: int, n: int, ncand: int) -> float:
    """Algorithmic FLOPs of exhaustive scoring per location: at design size j
    the contraction K_j^{-1} [k_c] over the ncand - j remaining candidates,
    2 j^2 (ncand - j)."""
    return float(sum(2.0 * j * j * (ncand - j) for j in range(n0, n)))


def time_steps(fn, steps: int, events_per_step: int):
    """Run fn(ev) steps times; fn records events_per_step+1 torch events on the
    current stream.  Returns per-phase mean ms and total wall ms."""
    import torch

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(events_per_step + 1)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        fn(evs[s])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    phases = np.array([[evs[s][k].elapsed_time(evs[s][k + 1]) for k in range(events_per_step)] for s in range(steps)])
    return phases.mean(axis=0), wall


def cpu_baseline(w, params, target_s: float = 15.0):
    """The oracle on the host cores over a bounded sample of the same
    locations, sized to take about target_s seconds."""
    import oracle

    cores = len(os.sched_getaffinity(0))
    probe = min(w.XX.shape[0], max(cores, 8))
    t0 = time.perf_counter()
    oracle.predict(w.X, w.y, w.XX[:probe], params, nthreads=cores)
    dt = time.perf_counter() - t0
    m = int(min(w.XX.shape[0], max(probe, probe * target_s / max(dt, 1e-3))))
    m = max(cores, (m // cores) * cores)
    t0 = time.perf_counter()
    oracle.predict(w.X, w.y, w.XX[:m], params, nthreads=cores)
    dt = time.perf_counter() - t0
    return dict(value=m / dt, unit="predictions/s", cores=cores, kind="oracle",
                sample=f"first {m} of the {w.XX.shape[0]} locations, {dt:.1f} s, OpenMP over locations")


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--M", type=int, default=None, help="fewer predictive locations (smoke runs)")
    ap.add_argument("--ray-steps", type=int, default=2)
    ap.add_argument("--no-ray", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the path is data parallel over locations and this build runs on a "
              "single MI355X; --gpus must be 1", file=sys.stderr)
        return 2

    import torch

    import paper_1409_0074_amd as lg
    from paper_1409_0074_amd import workloads as W

    lg.lib()
    w = W.uniform8d(M=args.M, search=W.SEARCH_EXHAUSTIVE)
    prm = w.params
    M, nc = w.XX.shape[0], prm.ncand
    dev = torch.device("cuda:0")
    X = torch.from_numpy(w.X).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    XX = torch.from_numpy(w.XX).to(dev)
    design = lg.lagp_design_create(X, y)
    P = lg.make_params(prm)
    cand = torch.empty((M, nc), dtype=torch.int32, device=dev)
    f64 = dict(dtype=torch.float64, device=dev)
    mean, s2, df = torch.empty(M, **f64), torch.empty(M, **f64), torch.empty(M, **f64)
    status = torch.empty(M, dtype=torch.int32, device=dev)
    sel = torch.empty((M, prm.n), dtype=torch.int32, device=dev)

    def step(ev, P=P, sel_out=None):
        ev[0].record()
        lg.lagp_candidates(design, XX, nc, cand)
        ev[1].record()
        lg.lagp_predict_candidates(design, XX, cand, P, mean, s2, df, sel_out, None, status)
        ev[2].record()

    dummy = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    for _ in range(args.warmup):
        step(dummy, sel_out=sel)
    torch.cuda.synchronize()
    ex_sel = sel.cpu().numpy().copy()
    ex_mean = mean.cpu().numpy().copy()
    (t_knn, t_local), wall = time_steps(step, args.steps, 2)
    ms_step = wall / args.steps
    value = M / (ms_step / 1e3)
    st = status.cpu().numpy()

    flops = scoring_flops(prm.n0, prm.n, nc) * M
    achieved = flops / (t_local / 1e3) / 1e12
    result = {
        "metric": "local-GP predictions/sec at N=1e6, n=50 (exhaustive vs ray); p99 latency",
        "value": round(value, 2),
        "unit": "predictions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "N": int(w.X.shape[0]), "p": 8, "M": M, "n0": prm.n0, "n": prm.n,
                   "ncand": nc, "search": "exhaustive", "kernel": "separable gaussian, d=0.5, g=1e-6",
                   "parallelism": "one GPU, data parallel over locations"},
        "phases_ms": {"knn": round(float(t_knn), 3), "local_design": round(float(t_local), 3)},
        "roofline": {"bound": "mfma", "kernel": "k_local (exhaustive scoring)", "achieved": round(achieved, 3),
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                     "traffic": None,
                     "work": f"sum_j 2 j^2 (ncand - j), j = n0..n-1: {scoring_flops(prm.n0, prm.n, nc):.4g} "
                             f"FLOP/location x {M} locations per launch"},
        "status_nonzero": int((st != 0).sum()),
    }

    if not args.no_ray:
        Pr = lg.make_params(prm, search=W.SEARCH_RAY, numrays=10)

        def rstep(ev):
            step(ev, P=Pr)

        rstep(dummy)
        torch.cuda.synchronize()
        (rk, rl), rwall = time_steps(rstep, args.ray_steps, 2)
        rms = rwall / args.ray_steps
        ry_mean = mean.cpu().numpy()
        rmse = lambda a: float(np.sqrt(np.mean((a - w.truth) ** 2)))  # noqa: E731
        result["ray"] = {"value": round(M / (rms / 1e3), 2), "unit": "predictions/s", "ms_per_step": round(rms, 3),
                         "numrays": 10, "phases_ms": {"knn": round(float(rk), 3), "local_design": round(float(rl), 3)},
                         "rmse_vs_truth": rmse(ry_mean), "exhaustive_rmse_vs_truth": rmse(ex_mean),
                         "rmse_ray_vs_exhaustive": float(np.sqrt(np.mean((ry_mean - ex_mean) ** 2)))}

    lg.lagp_design_destroy(design)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(w, prm)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
