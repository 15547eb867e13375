"""Local designs past 128 points (up to n = 256) against the oracle, bit for
bit (MI355X only): ray and nearest-neighbour searches with K_J^{-1} in a
per-location workspace, exhaustive search by streamed Cholesky columns, and
local MLE with the likelihood's matrices in a workspace (one and two
stages).  The shapes of the n = 200 rows of Table 1 (Sec. 5.1) included."""
import numpy as np
import pytest

import oracle
from paper_1409_0074_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lg():
    import torch

    import paper_1409_0074_amd as lg

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lg.lib()
    return lg


def _uniform(seed, N, p, M, **kw):
    rng = np.random.default_rng(seed)
    X = rng.random((N, p))
    y = np.sin(3.0 * X).sum(axis=1) + X[:, 0] * X[:, -1]
    return W.Workload(f"u{p}", X, y, rng.random((M, p)), W.Params(**kw))


def _run(lg, w, prm, mle_mode=0):
    import torch

    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    try:
        if mle_mode:
            out = d.predict_mle(torch.from_numpy(w.XX), prm, mode=mle_mode)
        else:
            out = d.predict(torch.from_numpy(w.XX), prm, diag=prm.search != W.SEARCH_NN)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    finally:
        d.close()


def _same(g, o, keys, what):
    for k in keys:
        assert np.array_equal(g[k], o[k], equal_nan=True), (what, k, np.argwhere(g[k] != o[k])[:3])


KEYS = ("sel", "mean", "s2", "status")


@pytest.mark.parametrize("p,R,n,snap", [
    (2, 1, 200, W.SNAP_DESIGN),      # the Table 1 ray rows' shape (one ray, the whole design)
    (2, 2, 200, W.SNAP_CANDIDATES),
    (3, 3, 130, W.SNAP_CANDIDATES),  # just past 128 points
    (4, 4, 256, W.SNAP_DESIGN),      # the largest n
])
def test_rays_past_128_points(lg, p, R, n, snap):
    w = _uniform(950 + p + n, 30000, p, 4, n0=6, n=n, search=W.SEARCH_RAY, numrays=R, d=(0.05 * p,), g=1e-6,
                 snap=snap)
    prm = w.params.replace(ncand=W.ray_candidates_needed(n, 6, R) + (0 if snap == W.SNAP_DESIGN else 300))
    g = _run(lg, w, prm)
    o = oracle.predict(w.X, w.y, w.XX, prm)
    _same(g, o, KEYS, f"rays p={p} R={R} n={n}")
    assert np.array_equal(g["diag"][:, :, 0], o["diag"][:, :, 1])


@pytest.mark.parametrize("n", [129, 200])
def test_nearest_neighbours_past_128_points(lg, n):
    w = _uniform(960 + n, 20000, 2, 5, n0=6, n=n, ncand=n, search=W.SEARCH_NN, d=(0.1,), g=1e-6)
    _same(_run(lg, w, w.params), oracle.predict(w.X, w.y, w.XX, w.params), KEYS, f"nn n={n}")


def test_cholesky_columns_at_n200(lg):
    w = _uniform(970, 30000, 2, 4, n0=6, n=200, ncand=1200, d=(0.1,), g=1e-6, scoring=W.SCORING_CHOL)
    g = _run(lg, w, w.params)
    o = oracle.predict(w.X, w.y, w.XX, w.params)
    _same(g, o, KEYS, "chol n=200")
    assert np.array_equal(g["diag"][:, :, 0], o["diag"][:, :, 1])


@pytest.mark.parametrize("search,n,mode", [
    (W.SEARCH_RAY, 200, 2),   # Table 1: ray, n = 200, two stages
    (W.SEARCH_RAY, 200, 1),   # ray, n = 200, one stage
    (W.SEARCH_NN, 200, 1),    # nn, n = 200
    (W.SEARCH_EXHAUSTIVE, 80, 2),  # between the LDS sizes and 128 (Cholesky columns streamed)
])
def test_local_mle_past_50_points(lg, search, n, mode):
    w = W.paper2d(M=6, n=n, search=search, numrays=1)
    prm = w.params
    if search == W.SEARCH_RAY:
        prm = prm.replace(ncand=W.ray_candidates_needed(n, 6, 1), snap=W.SNAP_DESIGN)
    elif search == W.SEARCH_NN:
        prm = prm.replace(ncand=n)
    g = _run(lg, w, prm, mle_mode=mode)
    o = oracle.predict_mle(w.X, w.y, w.XX, prm, mode=mode)
    _same(g, o, ("sel", "mean", "s2", "dhat", "iters", "status"), f"mle {search} n={n} mode={mode}")


def test_large_designs_are_checked(lg):
    import torch

    w = _uniform(980, 3000, 2, 2, n0=6, n=129, ncand=500, d=(0.1,), g=1e-6)
    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    try:
        for prm in (w.params, w.params.replace(precision=W.PREC_MIXED), w.params.replace(n=257, ncand=600)):
            with pytest.raises(lg.LagpError):  # partitioned inverse / mixed past 128 points; n > 256
                d.predict(torch.from_numpy(w.XX), prm)
    finally:
        d.close()
