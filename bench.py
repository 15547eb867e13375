#!/usr/bin/env python3
"""Local approximate GP prediction throughput on one MI355X.

One step = the whole hot path over the predictive set of the uniform 8-d
workload (N = 1e6 design points, M = 1e4 locations, n = 50, 1000 nearest
candidates, exhaustive greedy ALC search): candidate kNN, then the local
design search (criterion scored through incremental Cholesky columns) and
prediction.  Inputs are resident in HBM before timing starts.  The
partitioned-inverse scoring form and the ray-search form (10 rays) run on the
same inputs and are reported beside it, as is the CPU oracle on a bounded
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

# HBM traffic of one launch of each local-design kernel over the uniform 8-d
# workload (M = 1e4), from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE)
# of `bench.py --steps 1 --warmup 0 --ray-steps 1 --no-cpu --no-serving --no-mle
# --no-ray-sweep --no-sec51 --no-prescale --no-grid --copy-calibration-mb 1024`, each scaled by what the counter
# read for a 1 GiB device copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  Valid only for the kernel sources it was
# taken on (sha256); otherwise reported as null.
COMMON_SOURCES = ("paper_1409_0074_amd/csrc/dev_math.h", "paper_1409_0074_amd/csrc/lagp_internal.h",
                  "paper_1409_0074_amd/csrc/api.cpp")
KERNEL_SOURCES = {"k_chol": ("paper_1409_0074_amd/csrc/chol.hip",) + COMMON_SOURCES,
                  "k_local": ("paper_1409_0074_amd/csrc/local.hip",) + COMMON_SOURCES,
                  "k_local_ray": ("paper_1409_0074_amd/csrc/local.hip",) + COMMON_SOURCES}
MEASURED_TRAFFIC = {
    "k_chol": {"sha256": "e33583570e7db6089256086d368046d00b7833ca4c73692c84b1abc541b49eb1",
               "bytes": 2.3422e+09, "fetch_kib": 1123071.4, "write_kib": 41193.2},
    "k_local": {"sha256": "d0b3810627f7f6e1fbfd78f97dedb74acc1a5a6c53d83bc9925e45781f9b34f4",
                "bytes": 1.4054e+11, "fetch_kib": 66332140.9, "write_kib": 4578604.7},
    "k_local_ray": {"sha256": "d0b3810627f7f6e1fbfd78f97dedb74acc1a5a6c53d83bc9925e45781f9b34f4",
                    "bytes": 2.1522e+10, "fetch_kib": 10141631.9, "write_kib": 734717.2},
}


def kernel_sources_sha256(kernel: str) -> str:
    import hashlib

    h = hashlib.sha256()
    here = os.path.dirname(os.path.abspath(__file__))
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(here, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel: str, M: int):
    t = MEASURED_TRAFFIC.get(kernel)
    if t is None or M != 10000 or t["sha256"] != kernel_sources_sha256(kernel):
        return None
    return t["bytes"]


def scoring_bytes(n0: int, n: int, ncand: int) -> float:
    """Algorithmic bytes of exhaustive scoring per location: at design size j
    the j kernel-row entries of each of the ncand - j remaining candidates
    are read once, 8 j (ncand - j)."""
    return float(sum(8.0 * j * (ncand - j) for j in range(n0, n)))


def scoring_flops(n0: int, n: int, ncand: int) -> float:
    """Algorithmic FLOPs of exhaustive scoring per location: at design size j
    the contraction K_j^{-1} [k_c] over the ncand - j remaining candidates,
    2 j^2 (ncand - j)."""
    return float(sum(2.0 * j * j * (ncand - j) for j in range(n0, n)))


def chol_flops(n0: int, n: int, ncand: int, p: int) -> float:
    """FLOPs of the Cholesky-column search per location, counting the
    arithmetic each candidate does: after design point j is taken, the
    ncand - j - 1 free candidates each run the length-j inner product
    (2 j), the kernel value (4 p for the weighted squared distance, 34 for
    exp: the reduction and the degree-13 Horner polynomial), the new entry
    (2) and the updates of v, cov and q (6); every search step scores the
    ncand - j free candidates (2: a square and a division)."""
    upd = sum((ncand - j - 1) * (2.0 * j + 4 * p + 34 + 2 + 6) for j in range(n - 1))
    score = sum(2.0 * (ncand - j) for j in range(n0, n))
    return float(upd + score)


def chol_alg_flops(n0: int, n: int, ncand: int, p: int) -> float:
    """Algorithmic FLOPs of the Cholesky-column search per location: after
    design point j is taken, each of the ncand - j - 1 free candidates needs
    the length-j inner product u_t^T u_c (2 j) and the kernel value's
    weighted squared distance (3 p); exp is not counted."""
    return float(sum((ncand - j - 1) * (2.0 * j + 3.0 * p) for j in range(n - 1)))


def chol_stream_bytes(n: int, ncand: int) -> float:
    """Algorithmic device-memory bytes of the streamed Cholesky columns per
    location: after design point j is taken, each of the ncand - j - 1 free
    columns is read (j entries) and gains one entry, 8 (j + 1) bytes."""
    return float(sum(8.0 * (j + 1) * (ncand - j - 1) for j in range(n - 1)))


def ray_flops(evals, n0: int, ncand: int, p: int) -> float:
    """Work of the ray search from the Brent evaluations each step actually
    made (evals: locations x steps, summed over the step's rays): an
    evaluation at design size j costs j kernel values (3 p + 20: distance and
    exp), K^{-1} k_z (2 j^2) and the two inner products (4 j); each step adds
    the snap's 3 p N' distance FLOPs."""
    j = n0 + np.arange(evals.shape[1], dtype=np.float64)
    per_eval = 2.0 * j * j + j * (3.0 * p + 20.0) + 4.0 * j
    return float((evals * per_eval[None, :]).sum() + evals.size * 3.0 * p * ncand)


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


def serving(nreq: int):
    """Serving workload: resident 4-d design (N = 2e6), requests of 1..1000
    locations (log-uniform), n from {30, 50, 100}, exhaustive or ray search,
    a quarter of the exhaustive ones in the mixed form; saturation
    throughput from a burst, then open-loop Poisson arrivals at half of it."""
    import torch

    import paper_1409_0074_amd as lg
    from paper_1409_0074_amd import loadgen
    from paper_1409_0074_amd import workloads as W

    w = W.serving4d()
    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    base = w.params
    budget, slots = 16 << 30, 8
    reqs = W.serving_requests(nreq, qps=1.0, precision_mix=0.25)
    mean_m = float(np.mean([r.XX.shape[0] for r in reqs]))
    loadgen.run(d.handle, reqs[:20], base, budget, slots, burst=True)  # warm-up
    sat = loadgen.run(d.handle, reqs, base, budget, slots, burst=True)
    qps = 0.5 * sat["pred_per_s"] / mean_m
    op = loadgen.run(d.handle, reqs, base, budget, slots, time_scale=1.0 / qps)
    d.close()
    return {"workload": w.name, "requests": nreq, "mean_locations": round(mean_m, 1),
            "saturation_pred_per_s": round(sat["pred_per_s"], 1), "qps": round(qps, 2),
            "p50_ms": round(op["p50_ms"], 3), "p99_ms": round(op["p99_ms"], 3),
            "pred_per_s": round(op["pred_per_s"], 1), "errors": len(op["errors"]) + len(sat["errors"]),
            "arrivals": "open-loop Poisson at half the burst throughput", "mixed_share_of_exhaustive": 0.25,
            "budget_bytes": budget, "slots": slots}


FP32_PEAK_TFLOPS = 157.3  # MI355X dense FP32 (matrix)


def grid_leg(M_chol: int, M_sub: int, steps: int):
    """The grid workload: a 1000 x 1000 grid design on [0,1]^2 (N = 1e6) with
    the 2-d bump response, n = 100, N' = 4000, d = 0.05, g = 1e-6,
    exhaustive search.  FP64 by Cholesky columns streamed from a device
    workspace over M_chol locations (1e5: the whole predictive set); the
    partitioned-inverse FP64 form and the mixed form (certified FP32 screen,
    FP64 re-score) over the first M_sub of them.  Each with the roofline of
    its search kernel (time from events around the search alone)."""
    import torch

    import paper_1409_0074_amd as lg
    from paper_1409_0074_amd import workloads as W

    w = W.grid2d(M=M_chol)
    prm = w.params
    n0, n, nc = prm.n0, prm.n, prm.ncand
    dev = torch.device("cuda:0")
    X = torch.from_numpy(w.X).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    XX = torch.from_numpy(w.XX).to(dev)
    design = lg.lagp_design_create(X, y)
    f64 = dict(dtype=torch.float64, device=dev)
    out = {"workload": f"grid2d_N1000000_n100_cand4000", "M_cholesky": M_chol, "M_partitioned_and_mixed": M_sub,
           "rows": {}}
    res = {}
    for tag, M, kw in (("fp64_cholesky", M_chol, dict(scoring=W.SCORING_CHOL)),
                       ("fp64_partitioned_inverse", M_sub, {}),
                       ("mixed", M_sub, dict(precision=W.PREC_MIXED))):
        P = lg.make_params(prm, **kw)
        XXm = XX[:M]
        cand = torch.empty((M, nc), dtype=torch.int32, device=dev)
        mean, s2, df = torch.empty(M, **f64), torch.empty(M, **f64), torch.empty(M, **f64)
        status = torch.empty(M, dtype=torch.int32, device=dev)
        sel = torch.empty((M, n), dtype=torch.int32, device=dev)
        counts = torch.empty((M, n - n0, 2), dtype=torch.int32, device=dev)

        def gstep(ev):
            ev[0].record()
            lg.lagp_candidates(design, XXm, nc, cand)
            ev[1].record()
            lg.lagp_predict_counts(design, XXm, cand, P, mean, s2, df, sel, None, status, counts)
            ev[2].record()

        lg.lagp_predict(design, XXm[:64], P, mean[:64], s2[:64], df[:64])  # warm-up
        torch.cuda.synchronize()
        (tk, tl), wall = time_steps(gstep, steps, 2)
        ms = wall / steps
        row = {"M": M, "pred_per_s": round(M / (ms / 1e3), 1), "ms_per_step": round(ms, 3),
               "phases_ms": {"knn": round(float(tk), 3), "local_design": round(float(tl), 3)},
               "status_nonzero": int((status != 0).sum().cpu())}
        if tag == "fp64_cholesky":
            b = chol_stream_bytes(n, nc) * M
            gbs = b / (tl / 1e3) / 1e9
            row["roofline"] = {"bound": "hbm", "kernel": "k_cholw (Cholesky columns streamed from a workspace)",
                               "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                               "work": f"sum_j 8 (j + 1)(ncand - j - 1) = {chol_stream_bytes(n, nc):.4g} "
                                       f"B/location x {M} locations per launch"}
        else:
            fl = scoring_flops(n0, n, nc) * M
            tf = fl / (tl / 1e3) / 1e12
            if tag == "mixed":
                ct = counts.cpu().numpy()
                tiles = (nc + 15) // 16
                free = nc - (n0 + np.arange(n - n0))
                row["certified_shortlist"] = {
                    "candidates_mean": round(float(ct[:, :, 0].mean()), 1),
                    "candidates_max": int(ct[:, :, 0].max()),
                    "fraction_of_free_candidates": round(float((ct[:, :, 0] / free[None, :]).mean()), 4),
                    "tiles_rescored_fraction": round(float(ct[:, :, 1].mean() / tiles), 4)}
                row["roofline"] = {"bound": "mfma", "kernel": "k_local (mixed: FP32 screen + FP64 re-score)",
                                   "achieved": round(tf, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                   "frac": round(tf / FP32_PEAK_TFLOPS, 4), "traffic": None,
                                   "work": f"sum_j 2 j^2 (ncand - j) = {scoring_flops(n0, n, nc):.4g} FLOP/location "
                                           f"(the screen's contraction) x {M} locations per launch"}
            else:
                row["roofline"] = {"bound": "mfma", "kernel": "k_local (exhaustive, partitioned inverse)",
                                   "achieved": round(tf, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                   "frac": round(tf / FP64_PEAK_TFLOPS, 4), "traffic": None,
                                   "work": f"sum_j 2 j^2 (ncand - j) = {scoring_flops(n0, n, nc):.4g} FLOP/location "
                                           f"x {M} locations per launch (16.6 FLOP/B: above the FP64 ridge)"}
        out["rows"][tag] = row
        res[tag] = {"sel": sel[:M_sub].cpu().numpy(), "mean": mean[:M_sub].cpu().numpy(),
                    "s2": s2[:M_sub].cpu().numpy()}
        del cand, counts
    lg.lagp_design_destroy(design)
    floor = 1e-6 * np.sqrt(np.mean(w.y ** 2))

    def agree(a, b):
        e_mu = np.abs(a["mean"] - b["mean"]) / np.maximum(np.abs(b["mean"]), floor)
        e_s2 = np.abs(a["s2"] - b["s2"]) / np.abs(b["s2"])
        return {"identical_designs": float(np.mean(np.all(a["sel"] == b["sel"], axis=1))),
                "mean_relerr_max": float(e_mu.max()), "s2_relerr_max": float(e_s2.max()),
                "mean_within_1e-5": float(np.mean(e_mu <= 1e-5)), "s2_within_1e-5": float(np.mean(e_s2 <= 1e-5))}

    out["mixed_vs_fp64_partitioned"] = agree(res["mixed"], res["fp64_partitioned_inverse"])
    out["fp64_partitioned_vs_cholesky"] = agree(res["fp64_partitioned_inverse"], res["fp64_cholesky"])
    return out


# Table 1 of Sec. 5.1 (left: 2010 iMac, 8 threads; right: 16 Sandy Bridge
# threads with two M2090 GPUs for the exhaustive search), seconds for the
# 9801 predictive locations: context beside this GPU's times, not a target.
SEC51_PAPER_SECS = {"ray_n200_stage2": 2948.9, "ray_n200_stage1": 1695.4, "nn_n200": 710.3,
                    "ray_n50_stage2": 87.8, "ext_n50_stage2": 436.8, "ray_n50_stage1": 45.6,
                    "ext_n50_stage1": 390.4, "nn_n50": 11.5}
SEC51_PAPER_RIGHT = {"ext_n50_cand1000_stage1": {"cpu_gpu": 91, "imac_rays": 46},
                     "ext_n50_cand2000_stage1": {"cpu_gpu": 120, "imac_rays": 46},
                     "ext_n128_cand2000_stage1": {"cpu_gpu": 590, "imac_rays": 377}}


def sec51(steps: int):
    """The 2-d experiment of Sec. 5.1 (Table 1's rows at n = 200 and n = 50,
    and the right-hand table's n = 128, N' = 2000): every design search
    coupled with local MLE of the lengthscale, one and two stages, over the
    99 x 99 predictive grid.
    Times cover the neighbour search, the designs, the fits and the
    predictions of all 9801 locations (inputs resident on the GPU)."""
    import torch
    from scipy.stats import t as student_t

    import paper_1409_0074_amd as lg
    from paper_1409_0074_amd import workloads as W

    w = W.paper2d()
    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    XX = torch.from_numpy(w.XX).cuda()
    # ray searches snap over the whole design (Sec. 5: no N' limit on them),
    # so their candidate lists only hold the starts' ranks; one row keeps the
    # N' = 1000 scope for comparison
    nray = W.ray_candidates_needed(50, w.params.n0, 1)
    nray200 = W.ray_candidates_needed(200, w.params.n0, 1)
    rows = [("ray_n200_stage2", W.SEARCH_RAY, 2, nray200, W.SCORING_PARTINV),
            ("ray_n200_stage1", W.SEARCH_RAY, 1, nray200, W.SCORING_PARTINV),
            ("nn_n200", W.SEARCH_NN, 1, 1000, W.SCORING_PARTINV),
            ("ray_n50_stage2", W.SEARCH_RAY, 2, nray, W.SCORING_PARTINV),
            ("ext_n50_stage2", W.SEARCH_EXHAUSTIVE, 2, 1000, W.SCORING_CHOL),
            ("ray_n50_stage1", W.SEARCH_RAY, 1, nray, W.SCORING_PARTINV),
            ("ext_n50_stage1", W.SEARCH_EXHAUSTIVE, 1, 1000, W.SCORING_CHOL),
            ("nn_n50", W.SEARCH_NN, 1, 1000, W.SCORING_PARTINV),
            ("ext_n50_cand2000_stage1", W.SEARCH_EXHAUSTIVE, 1, 2000, W.SCORING_CHOL),
            ("ray_n50_stage1_snap_cand1000", W.SEARCH_RAY, 1, 1000, W.SCORING_PARTINV),
            ("ext_n128_cand2000_stage1", W.SEARCH_EXHAUSTIVE, 1, 2000, W.SCORING_CHOL)]
    out = {"workload": w.name.replace("_exhaustive", ""), "M": int(w.XX.shape[0]), "d0": w.params.d[0],
           "g": w.params.g, "numrays": 1, "paper_secs_context": SEC51_PAPER_SECS,
           "paper_right_table_secs_context": SEC51_PAPER_RIGHT, "rows": {}}
    for name, search, mode, nc, scoring in rows:
        full = search == W.SEARCH_RAY and "snap_cand" not in name
        n = int(name.split("_n")[1].split("_")[0])
        prm = w.params.replace(n=n, search=search, numrays=1 if search == W.SEARCH_RAY else 0, ncand=nc,
                               scoring=scoring if search == W.SEARCH_EXHAUSTIVE else W.SCORING_PARTINV,
                               snap=W.SNAP_DESIGN if full else W.SNAP_CANDIDATES)
        d.predict_mle(XX[:256], prm, mode)
        torch.cuda.synchronize()
        reps = steps if n <= 50 else 1  # (the larger designs run seconds each)
        t0 = time.perf_counter()
        for _ in range(reps):
            o = d.predict_mle(XX, prm, mode)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        mu, s2 = o["mean"].cpu().numpy(), o["s2"].cpu().numpy()
        df = o["df"].cpu().numpy()
        half = student_t.ppf(0.975, df) * np.sqrt(s2)
        out["rows"][name] = {
            "seconds": round(dt, 4), "pred_per_s": round(w.XX.shape[0] / dt, 1),
            "rmse": float(np.sqrt(np.mean((mu - w.truth) ** 2))), "sd_mean": float(np.mean(np.sqrt(s2))),
            "coverage95": float(np.mean(np.abs(w.truth - mu) <= half)),
            "dhat_median": float(np.median(o["dhat"].cpu().numpy())),
            "likelihood_evaluations_mean": float(o["iters"].float().mean().cpu()),
            "status_nonzero": int((o["status"] != 0).sum().cpu()), "n": n, "ncand": nc,
            "snap": "whole design" if full else ("candidates" if search == W.SEARCH_RAY else None)}
    d.close()
    return out


def prescale_leg(steps: int, ns: int = 256):
    """Pre-scaling by global separable lengthscales (Sec. 5.3) on the
    anisotropic 8-d workload (N = 1e6, M = 1e4): the fit on a subset of ns
    rows, the scaling of design and locations, then exhaustive and ray
    (p rays) search with two-stage local MLE on the scaled inputs, beside
    the same searches on the raw inputs."""
    import torch

    import paper_1409_0074_amd as lg
    from paper_1409_0074_amd import workloads as W

    w = W.aniso8d()
    N, p = w.X.shape
    M = w.XX.shape[0]
    X = torch.from_numpy(w.X).cuda()
    XX = torch.from_numpy(w.XX).cuda()
    y = torch.from_numpy(w.y).cuda()
    idx = torch.from_numpy(W.aniso8d_subset(N, ns)).cuda()
    XS, yS = X[idx].contiguous(), y[idx].contiguous()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    theta, evals, st = lg.lagp_fit_separable(XS, yS, w.params.g, 1.0, 1e-3, 100.0, 1e-4, 100, 8)
    fit_s = time.perf_counter() - t0
    Xs, XXs = torch.empty_like(X), torch.empty_like(XX)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lg.lagp_prescale(X, theta, Xs)
    lg.lagp_prescale(XX, theta, XXs)
    torch.cuda.synchronize()
    scale_ms = (time.perf_counter() - t0) * 1e3
    out = {"workload": w.name, "subset_rows": ns, "theta_hat": [round(float(t), 4) for t in theta],
           "fit_seconds": round(fit_s, 4), "fit_evaluations": evals, "fit_status": st,
           "prescale_ms": round(scale_ms, 3), "rows": {}}
    for tag, Xd, XXd, d0 in (("raw", X, XX, 0.5), ("prescaled", Xs, XXs, 1.0)):
        d = lg.Design(Xd, y)
        for sname, search, nr in (("exhaustive", W.SEARCH_EXHAUSTIVE, 0), ("rays8", W.SEARCH_RAY, p)):
            prm = w.params.replace(d=(d0,), search=search, numrays=nr,
                                   scoring=W.SCORING_CHOL if search == W.SEARCH_EXHAUSTIVE else W.SCORING_PARTINV)
            d.predict_mle(XXd[:256], prm, 2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                o = d.predict_mle(XXd, prm, 2)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            mu = o["mean"].cpu().numpy()
            out["rows"][f"{tag}_{sname}"] = {
                "ms": round(dt * 1e3, 3), "pred_per_s": round(M / dt, 1),
                "rmse": float(np.sqrt(np.mean((mu - w.truth) ** 2))),
                "dhat_median": float(np.median(o["dhat"].cpu().numpy())),
                "status_nonzero": int((o["status"] != 0).sum().cpu())}
        d.close()
    return out


def ray_sweep(w, steps: int, counts):
    """Rays per greedy step R = 1..p on the 8-d workload (fixed d, the same
    candidates): rate of the design search and accuracy against the truth,
    beside the exhaustive search's (Sec. 5.3 reports no gain beyond p rays)."""
    import torch

    import paper_1409_0074_amd as lg
    from paper_1409_0074_amd import workloads as W

    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    XX = torch.from_numpy(w.XX).cuda()
    idx, _ = d.candidates(XX, w.params.ncand)
    M = XX.shape[0]
    out = {"workload": w.name.replace("_exhaustive", ""), "M": M, "rows": {}}
    f64 = dict(dtype=torch.float64, device="cuda")
    mean, s2, df = torch.empty(M, **f64), torch.empty(M, **f64), torch.empty(M, **f64)
    status = torch.empty(M, dtype=torch.int32, device="cuda")
    for R in counts:
        prm = w.params.replace(search=W.SEARCH_RAY, numrays=R) if R else w.params.replace(scoring=W.SCORING_CHOL)
        P = lg.make_params(prm)
        lg.lagp_predict_candidates(d.handle, XX[:256], idx[:256], P, mean[:256], s2[:256], df[:256], None, None,
                                   status[:256])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            lg.lagp_predict_candidates(d.handle, XX, idx, P, mean, s2, df, None, None, status)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        mu = mean.cpu().numpy()
        out["rows"][f"rays{R}" if R else "exhaustive"] = {
            "design_ms": round(dt * 1e3, 3), "pred_per_s": round(M / dt, 1),
            "rmse": float(np.sqrt(np.mean((mu - w.truth) ** 2))), "status_nonzero": int((status != 0).sum().cpu())}
    d.close()
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--M", type=int, default=None, help="fewer predictive locations (smoke runs)")
    ap.add_argument("--ray-steps", type=int, default=2)
    ap.add_argument("--no-ray", action="store_true")
    ap.add_argument("--no-mle", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=400)
    ap.add_argument("--no-sec51", action="store_true", help="skip the Sec. 5.1 2-d experiment (Table 1 rows)")
    ap.add_argument("--no-ray-sweep", action="store_true", help="skip the rays-per-step sweep R = 1..p")
    ap.add_argument("--no-prescale", action="store_true", help="skip the pre-scaling leg (anisotropic 8-d)")
    ap.add_argument("--no-grid", action="store_true", help="skip the 2-d grid workload (n = 100, N' = 4000)")
    ap.add_argument("--grid-M", type=int, default=100000, help="grid locations for the Cholesky FP64 form")
    ap.add_argument("--grid-M-sub", type=int, default=10000,
                    help="grid locations for the partitioned-inverse FP64 and mixed forms")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="first run 3 plain device-to-device copies of this many MiB (reference for HBM counters)")
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
    calib = None
    if args.copy_calibration_mb > 0:
        nbytes = args.copy_calibration_mb << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        calib = {"bytes_read": nbytes, "bytes_written": nbytes, "copies": 3}
        del src, dst
    w = W.uniform8d(M=args.M, search=W.SEARCH_EXHAUSTIVE)
    prm = w.params
    M, nc = w.XX.shape[0], prm.ncand
    dev = torch.device("cuda:0")
    X = torch.from_numpy(w.X).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    XX = torch.from_numpy(w.XX).to(dev)
    design = lg.lagp_design_create(X, y)
    P = lg.make_params(prm, scoring=W.SCORING_CHOL)
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
    (t_knn, t_local), wall = time_steps(step, args.steps, 2)
    ex_mean = mean.cpu().numpy().copy()  # (the last timed step's)
    ms_step = wall / args.steps
    value = M / (ms_step / 1e3)
    st = status.cpu().numpy()

    p = int(w.X.shape[1])
    cflops = chol_flops(prm.n0, prm.n, nc, p)
    aflops = chol_alg_flops(prm.n0, prm.n, nc, p)
    achieved = aflops * M / (t_local / 1e3) / 1e12
    impl_tf = cflops * M / (t_local / 1e3) / 1e12
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
                   "ncand": nc, "search": "exhaustive", "scoring": "incremental cholesky columns",
                   "kernel": "separable gaussian, d=0.5, g=1e-6",
                   "parallelism": "one GPU, data parallel over locations"},
        "phases_ms": {"knn": round(float(t_knn), 3), "local_design": round(float(t_local), 3)},
        # the search state stays in registers and LDS (nothing streams from
        # HBM after the candidate gather), so the bound is the FP64 vector
        # rate: 256 CUs x 4 SIMDs x 16 FMA lanes x 2 x 2.4 GHz = 78.6 TF/s
        "roofline": {"bound": "alu", "kernel": "k_chol (exhaustive search, Cholesky scoring)",
                     "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": measured_traffic("k_chol", M),
                     "work": f"sum_j (ncand - j - 1)(2 j + 3 p) = {aflops:.4g} FLOP/location (the inner products "
                             f"u_t^T u_c and the kernel values' squared distances) x {M} locations per launch",
                     "implementation": {"achieved": round(impl_tf, 3), "frac": round(impl_tf / FP64_PEAK_TFLOPS, 4),
                                        "work": f"{cflops:.4g} FLOP/location (also exp as 34 FLOP, the new "
                                                f"entry, the updates of v, cov, q and the scores)"}},
        "status_nonzero": int((st != 0).sum()),
    }
    if calib is not None:
        result["copy_calibration"] = calib

    # the partitioned-inverse scoring form (the paper's update; FP64 MFMA
    # contraction over kernel rows streamed from HBM)
    Pp = lg.make_params(prm)

    def pstep(ev, sel_out=None):
        step(ev, P=Pp, sel_out=sel_out)

    pstep(dummy, sel_out=sel)
    torch.cuda.synchronize()
    pi_sel = sel.cpu().numpy().copy()
    pi_mean = mean.cpu().numpy().copy()
    (pk, pl), pwall = time_steps(pstep, args.ray_steps, 2)
    pms = pwall / args.ray_steps
    pflops = scoring_flops(prm.n0, prm.n, nc) * M
    pbytes = scoring_bytes(prm.n0, prm.n, nc) * M
    p_gbs = pbytes / (pl / 1e3) / 1e9
    p_tf = pflops / (pl / 1e3) / 1e12
    same = np.all(pi_sel == ex_sel, axis=1)
    result["partitioned_inverse"] = {
        "value": round(M / (pms / 1e3), 2), "unit": "predictions/s", "ms_per_step": round(pms, 3),
        "phases_ms": {"knn": round(float(pk), 3), "local_design": round(float(pl), 3)},
        # the candidate rows stream from HBM once per step: 8.3 FLOP/B, under
        # the FP64 ridge (78.6 TF/s / 8 TB/s = 9.8), so HBM is the bound
        "roofline": {"bound": "hbm", "kernel": "k_local (exhaustive, partitioned inverse)",
                     "achieved": round(p_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(p_gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic("k_local", M),
                     "work": f"sum_j 8 j (ncand - j), j = n0..n-1: {scoring_bytes(prm.n0, prm.n, nc):.4g} "
                             f"B/location x {M} locations per launch",
                     "mfma": {"achieved": round(p_tf, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                              "frac": round(p_tf / FP64_PEAK_TFLOPS, 4),
                              "work": f"sum_j 2 j^2 (ncand - j): {scoring_flops(prm.n0, prm.n, nc):.4g} "
                                      f"FLOP/location"}},
    }
    if args.warmup > 0:  # (the Cholesky form's designs come from its warm-up step)
        result["partitioned_inverse"].update({
            "identical_designs_vs_cholesky": float(np.mean(same)),
            "mean_relerr_max_vs_cholesky": float(np.max(np.abs(pi_mean[same] - ex_mean[same]) /
                                                        np.maximum(np.abs(ex_mean[same]), 1e-12), initial=0.0))})

    if not args.no_mle:
        # the paper's full local procedure (Sec. 5): local MLE of an isotropic
        # lengthscale and the two-stage re-design, on the same candidates
        Pm = lg.make_params(prm, d=(prm.d[0],), scoring=W.SCORING_CHOL)
        Qm = lg.make_mle_params(2)
        dhat = torch.empty(M, **f64)
        iters = torch.empty(M, dtype=torch.int32, device=dev)

        def mstep(ev):
            ev[0].record()
            lg.lagp_candidates(design, XX, nc, cand)
            ev[1].record()
            lg.lagp_predict_mle(design, XX, cand, Pm, Qm, mean, s2, df, dhat, None, iters, status)
            ev[2].record()

        mstep(dummy)
        torch.cuda.synchronize()
        (mk, ml), mwall = time_steps(mstep, args.ray_steps, 2)
        mms = mwall / args.ray_steps
        mm = mean.cpu().numpy()
        rmse = lambda a: float(np.sqrt(np.mean((a - w.truth) ** 2)))  # noqa: E731
        result["mle_two_stage"] = {
            "value": round(M / (mms / 1e3), 2), "unit": "predictions/s", "ms_per_step": round(mms, 3),
            "phases_ms": {"knn": round(float(mk), 3), "two_stage_designs_and_mle": round(float(ml), 3)},
            "d0": prm.d[0], "dhat_median": float(np.median(dhat.cpu().numpy())),
            "likelihood_evaluations_mean": float(iters.float().mean().cpu()),
            "status_nonzero": int((status != 0).sum().cpu()),
            "rmse_vs_truth": rmse(mm), "fixed_d_rmse_vs_truth": rmse(ex_mean)}

    if not args.no_ray:
        R = 10
        Pr = lg.make_params(prm, search=W.SEARCH_RAY, numrays=R)
        counts = torch.empty((M, prm.n - prm.n0, 2), dtype=torch.int32, device=dev)

        def rstep(ev):
            ev[0].record()
            lg.lagp_candidates(design, XX, nc, cand)
            ev[1].record()
            lg.lagp_predict_counts(design, XX, cand, Pr, mean, s2, df, None, None, status, counts)
            ev[2].record()

        rstep(dummy)
        torch.cuda.synchronize()
        (rk, rl), rwall = time_steps(rstep, args.ray_steps, 2)
        rms = rwall / args.ray_steps
        ry_mean = mean.cpu().numpy()
        ct = counts.cpu().numpy()
        ev_step, ev_ray_max = ct[:, :, 0].astype(np.float64), ct[:, :, 1]
        rflops = ray_flops(ev_step, prm.n0, nc, p)
        r_tf = rflops / (rl / 1e3) / 1e12
        rmse = lambda a: float(np.sqrt(np.mean((a - w.truth) ** 2)))  # noqa: E731
        result["ray"] = {
            "value": round(M / (rms / 1e3), 2), "unit": "predictions/s", "ms_per_step": round(rms, 3),
            "numrays": R, "phases_ms": {"knn": round(float(rk), 3), "local_design": round(float(rl), 3)},
            "rmse_vs_truth": rmse(ry_mean), "exhaustive_rmse_vs_truth": rmse(ex_mean),
            "rmse_ray_vs_exhaustive": float(np.sqrt(np.mean((ry_mean - ex_mean) ** 2))),
            "brent_evaluations": {"per_step_mean": round(float(ev_step.mean()), 2),
                                  "per_step_max": int(ev_step.max()),
                                  "per_ray_mean": round(float(ev_step.mean()) / R, 2),
                                  "per_ray_max": int(ev_ray_max.max()),
                                  "slowest_ray_over_mean_per_step": round(float((ev_ray_max / np.maximum(
                                      ev_step / R, 1e-9)).mean()), 3)},
            # Brent's iterations are short dependent chains of FP64 vector
            # work (kernel values, K^{-1} k_z, inner products): FP64 VALU bound
            "roofline": {"bound": "alu", "kernel": "k_local (ray search, 10 rays)", "achieved": round(r_tf, 3),
                         "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(r_tf / FP64_PEAK_TFLOPS, 4),
                         "traffic": measured_traffic("k_local_ray", M),
                         "work": f"sum over steps of E_j (2 j^2 + j (3 p + 20) + 4 j) + 3 p N' with E_j the "
                                 f"kernel's own Brent evaluations: {rflops / M:.4g} FLOP/location x {M} "
                                 f"locations per launch"}}

    if not args.no_ray:
        # the same rays snapping over the whole design (Sec. 5): the results
        # do not depend on the list length (at least the starts' ranks); the
        # 1000-nearest lists settle most snaps without the design's grid
        ncr = max(W.ray_candidates_needed(prm.n, prm.n0, R), prm.ncand)
        Pf = lg.make_params(prm, search=W.SEARCH_RAY, numrays=R, ncand=ncr, snap=W.SNAP_DESIGN)
        candr = torch.empty((M, ncr), dtype=torch.int32, device=dev)
        selr = torch.empty((M, prm.n), dtype=torch.int32, device=dev)
        lg.lagp_design_build_grid(design)

        def fstep(ev):
            ev[0].record()
            lg.lagp_candidates(design, XX, ncr, candr)
            ev[1].record()
            lg.lagp_predict_counts(design, XX, candr, Pf, mean, s2, df, selr, None, status, counts)
            ev[2].record()

        fstep(dummy)
        torch.cuda.synchronize()
        (fk, fl), fwall = time_steps(fstep, args.ray_steps, 2)
        fms = fwall / args.ray_steps
        fct = counts.cpu().numpy()[:, :, 0]
        # chosen rows outside each location's 1000 nearest (their ranks in the
        # N' = 1000 lists of the exhaustive run)
        sr, cd = selr.cpu().numpy(), cand.cpu().numpy()
        outside = int(sum(np.sum(~np.isin(sr[m], cd[m])) for m in range(0, M, 10)))
        result["ray"]["snap_design"] = {
            "value": round(M / (fms / 1e3), 2), "unit": "predictions/s", "ms_per_step": round(fms, 3),
            "ncand": ncr, "phases_ms": {"knn": round(float(fk), 3), "local_design": round(float(fl), 3)},
            "rmse_vs_truth": rmse(mean.cpu().numpy()),
            "brent_evaluations_per_step_mean": round(float(fct.mean()), 2),
            "rows_outside_1000_nearest": {"count": outside, "of": int(sr[::10].size), "sample": "every 10th location"},
            "status_nonzero": int((status != 0).sum().cpu())}

    lg.lagp_design_destroy(design)
    del X, y, XX, cand
    if not args.no_ray_sweep:
        result["ray_sweep"] = ray_sweep(w, args.ray_steps, [0] + list(range(1, w.X.shape[1] + 1)))
    if not args.no_sec51:
        result["sec51"] = sec51(args.ray_steps)
    if not args.no_prescale:
        result["prescale"] = prescale_leg(args.ray_steps)
    if not args.no_serving:
        result["serving"] = serving(args.serving_requests)
    if not args.no_grid:
        result["grid"] = grid_leg(args.grid_M, min(args.grid_M, args.grid_M_sub), 1)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(w, prm.replace(scoring=W.SCORING_CHOL))
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
