"""Open-loop load generator for the continuous-batching server.

Requests are submitted at their scheduled (Poisson) arrival times whether or
not earlier ones have finished, so queueing delay shows up in the latency
instead of slowing the arrivals down; a second thread fetches results.
Latency is the server's own submit-to-ready time.
"""
from __future__ import annotations

import threading
import time

import numpy as np

from . import (LAGP_EAGAIN, lagp_server_create, lagp_server_destroy, lagp_server_fetch, lagp_server_stats,
               lagp_server_submit, make_params)
from . import workloads as W


def request_params(base: W.Params, req: W.Request) -> W.Params:
    """A request's method parameters: exhaustive FP64 requests are scored by
    Cholesky columns (on chip up to n = 50 and N' = 1024, streamed from a
    workspace beyond), mixed-form requests by the partitioned-inverse form
    the mixed screen applies to."""
    ncand = max(base.ncand, req.n + 64)
    chol = req.search == W.SEARCH_EXHAUSTIVE and req.precision == W.PREC_FP64
    return base.replace(n=req.n, search=req.search, precision=req.precision, ncand=ncand,
                        scoring=W.SCORING_CHOL if chol else W.SCORING_PARTINV)


def run(design_handle, requests, base: W.Params, budget_bytes: int, max_inflight: int, time_scale: float = 1.0,
        burst: bool = False):
    """Serve `requests` (workloads.Request) and return a stats dict.  With
    burst=True every request is submitted at once (saturation throughput)."""
    srv = lagp_server_create(design_handle, budget_bytes, max_inflight)
    tickets = [None] * len(requests)
    ready = [threading.Event() for _ in requests]
    results = [None] * len(requests)
    errors = []

    def fetcher():
        for k, req in enumerate(requests):
            ready[k].wait()
            try:
                results[k] = lagp_server_fetch(srv, tickets[k], req.XX.shape[0], req.n)
            except Exception as e:  # pragma: no cover - reported below
                errors.append(repr(e))

    th = threading.Thread(target=fetcher, daemon=True)
    th.start()
    t0 = time.perf_counter()
    try:
        for k, req in enumerate(requests):
            if not burst:
                delay = t0 + req.arrival_s * time_scale - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            P = make_params(request_params(base, req))
            while True:
                rc, t = lagp_server_submit(srv, req.XX, P)
                if rc != LAGP_EAGAIN:
                    break
                time.sleep(1e-4)
            tickets[k] = t
            ready[k].set()
        th.join()
        wall = time.perf_counter() - t0
        st = lagp_server_stats(srv)
    finally:
        lagp_server_destroy(srv)
    lat = np.array([r["latency_ms"] for r in results if r is not None])
    preds = int(sum(r.XX.shape[0] for r in requests))
    return dict(requests=len(requests), predictions=preds, wall_s=wall, pred_per_s=preds / wall,
                p50_ms=float(np.percentile(lat, 50)) if lat.size else None,
                p99_ms=float(np.percentile(lat, 99)) if lat.size else None,
                server_p50_ms=st["p50_ms"], server_p99_ms=st["p99_ms"], errors=errors, results=results)
