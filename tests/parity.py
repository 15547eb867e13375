"""GPU-vs-oracle comparison helpers (test infrastructure).

The oracle always runs on its own inputs (it never receives a GPU result).
The FP64 forms of the library sum in the oracle's defined order, so their
designs and predictions are compared for bit equality; the mixed form is
compared run against run, and where its design departs from the FP64 one the
oracle's criterion value of the GPU's pick at that step is looked up in the
oracle's own trace of the location.
"""
from __future__ import annotations

import numpy as np

import oracle


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


def check_exact(w, params, g, XX=None, diag=True):
    """The GPU's run against the oracle's independent run of the same
    locations (the oracle never sees a GPU result): designs, means, scales
    and status words equal bit for bit, and the per-step best and runner-up
    criterion values too when the GPU reported them."""
    XX = w.XX if XX is None else XX
    o = oracle.predict(w.X, w.y, XX, params)
    assert np.array_equal(g["sel"], o["sel"]), f"designs differ at {np.argwhere(g['sel'] != o['sel'])[:3]}"
    assert np.array_equal(g["mean"], o["mean"], equal_nan=True)
    assert np.array_equal(g["s2"], o["s2"], equal_nan=True)
    assert np.array_equal(g["status"], o["status"])
    if diag and g.get("diag") is not None and params.search != 2 and params.n > params.n0:
        assert np.array_equal(g["diag"][:, :, 0], o["diag"][:, :, 1])
        assert np.array_equal(g["diag"][:, :, 1], o["diag"][:, :, 2])
    return o


def first_divergence(g_sel, o_sel):
    """Per location, the first design position where two selection
    sequences differ (-1 where they agree throughout)."""
    out = np.full(g_sel.shape[0], -1)
    for m in range(g_sel.shape[0]):
        d = np.nonzero(g_sel[m] != o_sel[m])[0]
        if d.size:
            out[m] = d[0]
    return out


def oracle_pick_value(w, params, m, step, row, XX=None):
    """The oracle's criterion value of design row `row` at greedy step
    `step` of its own run at location m (from its full trace)."""
    XX = w.XX if XX is None else XX
    tr = oracle.trace(w.X, w.y, XX[m], params)
    q = int(np.nonzero(tr["cand"] == row)[0][0])
    return tr["alc"][step - params.n0][q], tr["diag"][step - params.n0]
