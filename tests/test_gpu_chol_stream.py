"""Cholesky-column scoring past the on-chip sizes (columns streamed from a
device workspace) against the oracle's Cholesky form, bit for bit (MI355X
only).  The same kernel is forced onto small shapes through the test hook
LAGP_CHOL_FORCE_STREAM=1, where it must also equal the on-chip kernel."""
import numpy as np
import pytest

import oracle
from paper_1409_0074_amd import workloads as W
from tests.parity import run_gpu

pytestmark = pytest.mark.gpu

CHOL = W.SCORING_CHOL


@pytest.fixture(scope="module")
def lg():
    import torch

    import paper_1409_0074_amd as lg

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lg.lib()
    return lg


def _exact(w, prm, diag=True):
    g = run_gpu(w, prm, diag=diag)
    o = oracle.predict(w.X, w.y, w.XX, prm)
    assert np.array_equal(g["sel"], o["sel"]), f"designs differ at {np.argwhere(g['sel'] != o['sel'])[:3]}"
    assert np.array_equal(g["mean"], o["mean"], equal_nan=True)
    assert np.array_equal(g["s2"], o["s2"], equal_nan=True)
    assert np.array_equal(g["status"], o["status"])
    if diag and prm.n > prm.n0:
        assert np.array_equal(g["diag"][:, :, 0], o["diag"][:, :, 1])
        assert np.array_equal(g["diag"][:, :, 1], o["diag"][:, :, 2])
    return g, o


def test_stream_grid_workload_shape(lg):
    """The 1000 x 1000 grid, N' = 4000, n = 100, d = 0.05, g = 1e-6 (eight
    candidates per thread), 24 locations."""
    w = W.grid2d(M=24)
    g, _ = _exact(w, w.params.replace(scoring=CHOL))
    assert np.all(g["status"] == 0)


@pytest.mark.parametrize("p,n,n0,ncand,N", [
    (2, 128, 6, 4096, 30000),   # the largest n and N'
    (4, 100, 6, 1000, 60000),   # the served workload's n = 100 shape (four per thread)
    (16, 60, 6, 2100, 40000),   # the largest p, eight per thread, ragged N'
    (3, 51, 1, 1025, 20000),    # just past the on-chip sizes in both n and N'
    (2, 70, 70, 300, 5000),     # n0 = n: no greedy step
    (1, 80, 6, 80, 3000),       # N' = n: every candidate is taken
])
def test_stream_shapes(lg, p, n, n0, ncand, N):
    w = W.small_case(700 + p + n, N, p, 5, n0=n0, n=n, ncand=ncand, d=(0.3 * p,) * p, g=1e-6, scoring=CHOL)
    _exact(w, w.params, diag=n0 < n)


def test_stream_distinct_lengthscales(lg):
    rng = np.random.default_rng(701)
    X = rng.random((50000, 4))
    d4 = (0.2, 0.5, 1.0, 2.0)
    w = W.Workload("u4", X, W.f_mix4(X), rng.random((7, 4)),
                   W.Params(n0=6, n=100, ncand=1500, d=d4, g=1e-6, scoring=CHOL))
    _exact(w, w.params)


@pytest.mark.parametrize("M", [1, 7, 300])
def test_stream_forced_small_shapes_equal_on_chip(lg, monkeypatch, M):
    """The benchmark's local shape (p = 8, n = 50, N' = 1000) through the
    streaming kernel: equal to the on-chip kernel's run and to the oracle,
    for location counts below and above the number of resident workgroups
    (1 and 7, and 300, which each workgroup loops over)."""
    rng = np.random.default_rng(702)
    X = rng.random((40000, 8))
    w = W.Workload("u8", X, W.f_sines8(X), rng.random((M, 8)),
                   W.Params(n0=6, n=50, ncand=1000, d=(0.5,) * 8, g=1e-6, scoring=CHOL))
    on_chip = run_gpu(w, w.params)
    monkeypatch.setenv("LAGP_CHOL_FORCE_STREAM", "1")
    g, _ = _exact(w, w.params) if M <= 7 else (run_gpu(w, w.params), None)
    for k in ("sel", "mean", "s2", "status", "diag"):
        assert np.array_equal(g[k], on_chip[k]), k


def test_stream_forced_singular_start(lg, monkeypatch):
    """Duplicated design points and g = 0: NaN, the NOTPD bit and the n0
    nearest, as in the oracle."""
    monkeypatch.setenv("LAGP_CHOL_FORCE_STREAM", "1")
    X = np.repeat(np.random.default_rng(703).random((300, 2)), 2, axis=0)
    w = W.Workload("dup", X, W.f_bump2(X), X[:4].copy(), W.Params(n0=4, n=10, ncand=40, d=(0.1,), g=0.0,
                                                                 scoring=CHOL))
    g, _ = _exact(w, w.params, diag=False)
    assert np.all(np.isnan(g["mean"])) and np.all(g["status"] & lg.LAGP_STATUS_NOTPD)


def test_stream_counts(lg):
    w = W.grid2d(M=3)
    prm = w.params.replace(scoring=CHOL)
    import torch

    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    try:
        out = d.predict(torch.from_numpy(w.XX), prm, counts=True)
        torch.cuda.synchronize()
        ct = out["counts"].cpu().numpy()
    finally:
        d.close()
    free = prm.ncand - (prm.n0 + np.arange(prm.n - prm.n0))
    assert np.array_equal(ct[:, :, 0], np.broadcast_to(free, ct.shape[:2])) and np.all(ct[:, :, 1] == 0)
