"""GPU-vs-oracle comparison helpers (test infrastructure).

Replay protocol: the oracle follows the GPU's selection sequence step by step
and records its own choice, the two best criterion values and the value of
the GPU's pick.  A step where the oracle's relative top-two gap exceeds
GAP_TOL must have the same pick; a closer step is exempt but the GPU's pick
must still score within GAP_TOL of the best.  Mean and scale are then the
oracle's on the GPU's design.
"""
from __future__ import annotations

import numpy as np

import oracle

GAP_TOL = 1e-9        # selection must match where the top-two gap exceeds this (relative)
VALUE_RTOL = 1e-8     # mean and scale, FP64 form


def run_gpu(w, params, XX=None, sel=True, diag=True):
    import torch

    import paper_1409_0074_amd as lg

    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    try:
        out = d.predict(torch.from_numpy(w.XX if XX is None else XX), params, sel=sel, diag=diag)
        torch.cuda.synchronize()
        return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    finally:
        d.close()


def rel_err(a, b, floor):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def check_replay(w, params, g, XX=None, rtol=VALUE_RTOL, bit_exact_values=False):
    """Replay the GPU's selections in the oracle; returns a stats dict and
    asserts the protocol."""
    XX = w.XX if XX is None else XX
    o = oracle.predict(w.X, w.y, XX, params, forced=g["sel"])
    assert np.all(o["status"] < 0x100), "oracle could not replay the GPU sequence"
    n0 = params.n0
    dg = o["diag"]                      # M x steps x NDIAG
    gpu_pick = g["sel"][:, n0:].astype(float)
    own = dg[:, :, 0]
    alc1, alc2, alc_take = dg[:, :, 1], dg[:, :, 2], dg[:, :, 3]
    gap = dg[:, :, 4]
    decisive = gap > GAP_TOL
    mism = decisive & (own != gpu_pick)
    assert not mism.any(), f"{mism.sum()} decisive steps differ; first at {np.argwhere(mism)[0]}"
    exempt = ~decisive
    if exempt.any():
        ok = alc_take[exempt] >= alc1[exempt] * (1.0 - GAP_TOL)
        assert ok.all(), "an exempt step took a clearly worse candidate"
    floor_mu = 1e-6 * np.sqrt(np.mean(w.y ** 2))
    e_mu = rel_err(g["mean"], o["mean"], floor_mu)
    e_s2 = rel_err(g["s2"], o["s2"], 1e-300)
    assert np.all(e_mu <= rtol), f"mean rel err {e_mu.max()}"
    assert np.all(e_s2 <= rtol), f"s2 rel err {e_s2.max()}"
    if bit_exact_values:
        assert np.array_equal(g["mean"], o["mean"]) and np.array_equal(g["s2"], o["s2"])
    return dict(steps=int(gap.size), exempt=int(exempt.sum()), max_err_mu=float(e_mu.max()),
                max_err_s2=float(e_s2.max()), min_gap=float(gap.min()))

