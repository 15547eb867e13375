"""Full-size workloads in the launch configuration bench.py times, checked
against the oracle on a seeded sample of locations (MI355X only).

The GPU runs every location of the workload in one call sequence (kNN over
the whole design, then the local designs), exactly as the benchmark does;
the oracle recomputes a sample of those locations one by one from scratch
(its own kNN over the full design).  The FP64 path sums in the defined
order, so the sampled designs, means and scales must be identical."""
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


def _bench_calls(lg, w, prm):
    """lagp_candidates then lagp_predict_candidates over every location, on
    device-resident inputs (the benchmark's step)."""
    import torch

    dev = torch.device("cuda:0")
    M, nc = w.XX.shape[0], prm.ncand
    X = torch.from_numpy(w.X).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    XX = torch.from_numpy(w.XX).to(dev)
    design = lg.lagp_design_create(X, y)
    try:
        P = lg.make_params(prm)
        cand = torch.empty((M, nc), dtype=torch.int32, device=dev)
        f64 = dict(dtype=torch.float64, device=dev)
        mean, s2, df = torch.empty(M, **f64), torch.empty(M, **f64), torch.empty(M, **f64)
        status = torch.empty(M, dtype=torch.int32, device=dev)
        sel = torch.empty((M, prm.n), dtype=torch.int32, device=dev)
        lg.lagp_candidates(design, XX, nc, cand)
        lg.lagp_predict_candidates(design, XX, cand, P, mean, s2, df, sel, None, status)
        torch.cuda.synchronize()
        return {"cand": cand.cpu().numpy(), "mean": mean.cpu().numpy(), "s2": s2.cpu().numpy(),
                "df": df.cpu().numpy(), "sel": sel.cpu().numpy(), "status": status.cpu().numpy()}
    finally:
        lg.lagp_design_destroy(design)


def _sample(M, k, seed):
    return np.sort(np.random.default_rng(seed).choice(M, size=k, replace=False))


@pytest.mark.parametrize("search", [W.SEARCH_EXHAUSTIVE, W.SEARCH_RAY])
def test_uniform8d_full_size_sampled(lg, search):
    """N = 1e6, p = 8, all 1e4 locations, n = 50, N' = 1000; exhaustive and
    10 rays; 24 sampled locations recomputed by the oracle."""
    w = W.uniform8d(search=search)
    prm = w.params
    g = _bench_calls(lg, w, prm)
    assert np.all(g["status"] == 0)
    assert np.all(g["df"] == prm.n)
    idx = _sample(w.XX.shape[0], 24, 501 + search)
    oi, _ = oracle.knn(w.X, w.XX[idx], prm.ncand)
    assert np.array_equal(g["cand"][idx].astype(np.int64), oi)
    o = oracle.predict(w.X, w.y, w.XX[idx], prm)
    assert np.array_equal(g["sel"][idx], o["sel"])
    assert np.array_equal(g["mean"][idx], o["mean"]) and np.array_equal(g["s2"][idx], o["s2"])


def test_uniform8d_full_size_sampled_chol(lg):
    """The same full-size workload with Cholesky-column scoring, against the
    oracle's Cholesky form on 24 sampled locations, bit for bit."""
    w = W.uniform8d()
    prm = w.params.replace(scoring=W.SCORING_CHOL)
    g = _bench_calls(lg, w, prm)
    assert np.all(g["status"] == 0)
    assert np.all(g["df"] == prm.n)
    idx = _sample(w.XX.shape[0], 24, 507)
    o = oracle.predict(w.X, w.y, w.XX[idx], prm)
    assert np.array_equal(g["sel"][idx], o["sel"])
    assert np.array_equal(g["mean"][idx], o["mean"]) and np.array_equal(g["s2"][idx], o["s2"])


def test_uniform8d_full_size_two_stage_mle_sampled(lg):
    """Two-stage local MLE over all 1e4 locations of the full-size 8-d
    workload (isotropic d0 = 0.5), as the benchmark runs it; 8 sampled
    locations recomputed by the oracle, bit for bit."""
    import torch

    w = W.uniform8d()
    prm = w.params.replace(d=(0.5,), scoring=W.SCORING_CHOL)
    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    try:
        out = d.predict_mle(torch.from_numpy(w.XX), prm, 2)
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        d.close()
    assert np.all(np.isfinite(g["mean"]))
    idx = _sample(w.XX.shape[0], 8, 509)
    o = oracle.predict_mle(w.X, w.y, w.XX[idx], prm, 2)
    for k in ("sel", "dhat", "iters", "status", "mean", "s2"):
        assert np.array_equal(g[k][idx], o[k]), k


@pytest.mark.parametrize("search,mode", [(W.SEARCH_RAY, 2), (W.SEARCH_EXHAUSTIVE, 2), (W.SEARCH_NN, 1)])
def test_sec51_full_size_mle_sampled(lg, search, mode):
    """The Sec. 5.1 experiment as the benchmark runs it: the 201 x 201 grid
    design, all 9801 locations of the 99 x 99 predictive grid, n = 50, local
    MLE; 16 sampled locations recomputed by the oracle, bit for bit."""
    import torch

    w = W.paper2d(search=search)
    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    try:
        out = d.predict_mle(torch.from_numpy(w.XX), w.params, mode)
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        d.close()
    assert np.all(np.isfinite(g["mean"])) and np.all(g["s2"] > 0)
    idx = _sample(w.XX.shape[0], 16, 511 + search)
    o = oracle.predict_mle(w.X, w.y, w.XX[idx], w.params, mode)
    for k in ("sel", "dhat", "iters", "status", "mean", "s2"):
        assert np.array_equal(g[k][idx], o[k]), k


def test_grid2d_full_size_sampled(lg):
    """1000 x 1000 grid design, n = 100, N' = 4000, the first 2000 locations
    through lagp_predict (as the benchmark's grid leg), 6 sampled locations
    recomputed by the oracle."""
    import torch

    w = W.grid2d(M=2000)
    prm = w.params
    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    try:
        out = d.predict(torch.from_numpy(w.XX), lg.make_params(prm), diag=False)
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    finally:
        d.close()
    assert np.all(g["status"] == 0)
    idx = _sample(w.XX.shape[0], 6, 503)
    o = oracle.predict(w.X, w.y, w.XX[idx], prm)
    assert np.array_equal(g["sel"][idx], o["sel"])
    assert np.array_equal(g["mean"][idx], o["mean"]) and np.array_equal(g["s2"][idx], o["s2"])


def test_aniso8d_full_size_prescaled_mle_sampled(lg):
    """The pre-scaling leg as the benchmark runs it: the global fit on the
    256-row subset of the 1e6-row anisotropic 8-d design (bit for bit as the
    oracle's), the scaling of design and all 1e4 locations, then exhaustive
    search with two-stage local MLE on the scaled inputs; 6 sampled
    locations recomputed by the oracle on numpy's scaled arrays."""
    import torch

    w = W.aniso8d()
    N = w.X.shape[0]
    idx = W.aniso8d_subset(N)
    X = torch.from_numpy(w.X).cuda()
    XX = torch.from_numpy(w.XX).cuda()
    y = torch.from_numpy(w.y).cuda()
    th, it, st = lg.lagp_fit_separable(X[idx].contiguous(), y[idx].contiguous(), w.params.g, 1.0, 1e-3, 100.0,
                                       1e-4, 100, 8)
    th_o, it_o, st_o = oracle.sep_fit(w.X[idx], w.y[idx], w.params.g, 1.0, 1e-3, 100.0, 1e-4, 100, 8)
    assert np.array_equal(th, th_o) and it == it_o and st == st_o
    Xs, XXs = torch.empty_like(X), torch.empty_like(XX)
    lg.lagp_prescale(X, th, Xs)
    lg.lagp_prescale(XX, th, XXs)
    prm = w.params.replace(d=(1.0,))
    d = lg.Design(Xs, y)
    try:
        out = d.predict_mle(XXs, prm, 2)
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        d.close()
    s = np.sqrt(th)
    Xn, XXn = w.X / s, w.XX / s
    pick = _sample(w.XX.shape[0], 6, 513)
    o = oracle.predict_mle(Xn, w.y, XXn[pick], prm, 2)
    for k in ("sel", "dhat", "iters", "status", "mean", "s2"):
        assert np.array_equal(g[k][pick], o[k]), k
    assert np.sqrt(np.mean((g["mean"] - w.truth) ** 2)) < 1e-3
