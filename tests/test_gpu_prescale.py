"""Global separable fit on a subset and input pre-scaling vs the oracle
(MI355X only).

The fit kernel evaluates the likelihood and its derivatives in the
oracle's order (O9) and takes the same Newton and sweep decisions, so
estimates, evaluation counts and status bits must be equal bit for bit.
Pre-scaling is one IEEE division by a correctly rounded square root per
element, equal to numpy's.  The local path on pre-scaled inputs is then the
ordinary one, checked against the oracle run on numpy's scaled arrays."""
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


def _fit_both(lg, XS, yS, g, theta0, dmin, dmax, tol=1e-8, maxit=100, maxsweep=20):
    import torch

    th_g, it_g, st_g = lg.lagp_fit_separable(torch.from_numpy(XS).cuda(), torch.from_numpy(yS).cuda(), g, theta0,
                                             dmin, dmax, tol, maxit, maxsweep)
    th_o, it_o, st_o = oracle.sep_fit(XS, yS, g, theta0, dmin, dmax, tol, maxit, maxsweep)
    assert np.array_equal(th_g, th_o), (th_g, th_o)
    assert it_g == it_o and st_g == st_o
    return th_g, it_g, st_g


@pytest.mark.parametrize("n,p,seed", [(40, 1, 1), (64, 3, 2), (100, 8, 3), (129, 5, 4)])
def test_sepfit_matches_oracle(lg, n, p, seed):
    rng = np.random.default_rng(700 + seed)
    XS = rng.random((n, p))
    yS = W.f_aniso8(np.pad(XS, ((0, 0), (0, max(0, 8 - p)))))
    th, it, st = _fit_both(lg, XS, yS, 1e-6, 0.5, 1e-3, 100.0, tol=1e-6, maxsweep=6)
    print(f"n={n} p={p}: theta {np.round(th, 4)}, evaluations {it}, status {st}")


def test_sepfit_bounds_budget_and_singular(lg):
    """A narrow range (bound), a one-evaluation budget (maxit), and a subset
    with a repeated row and no nugget (K singular at every lengthscale)."""
    rng = np.random.default_rng(710)
    XS = rng.random((50, 3))
    yS = W.f_aniso8(np.pad(XS, ((0, 0), (0, 5))))
    _, _, st = _fit_both(lg, XS, yS, 1e-6, 0.5, 0.4, 0.6)
    assert st & lg.LAGP_STATUS_MLE_BOUND
    _, _, st = _fit_both(lg, XS, yS, 1e-6, 0.5, 1e-3, 100.0, maxit=1, maxsweep=1)
    assert st & lg.LAGP_STATUS_MLE_MAXIT
    XS2 = np.vstack([XS, XS[:1]])
    yS2 = np.append(yS, yS[0])
    _, _, st = _fit_both(lg, XS2, yS2, 0.0, 0.5, 1e-3, 100.0, maxit=5, maxsweep=2)
    assert st & lg.LAGP_STATUS_MLE_NOTPD


def test_sepfit_bench_subset(lg):
    """The benchmark's fit: 256 rows of the anisotropic 8-d design."""
    w = W.aniso8d(M=1, N=100_000)
    idx = W.aniso8d_subset(w.X.shape[0])
    th, it, st = _fit_both(lg, w.X[idx], w.y[idx], 1e-6, 1.0, 1e-3, 100.0, tol=1e-4, maxsweep=8)
    # the inert inputs x5..x8 reach the upper bound, the fast one stays short
    assert np.all(th[4:] >= 99.0) and th[0] < 1.0


def test_sepfit_largest_subset(lg):
    """n = 1024 rows (the maximum): one Newton step of one coordinate (the
    oracle's evaluation at this size takes about ten seconds), bit for bit."""
    rng = np.random.default_rng(730)
    XS = rng.random((1024, 2))
    yS = np.sin(3.0 * XS[:, 0]) + XS[:, 1] ** 2
    th, it, st = _fit_both(lg, XS, yS, 1e-6, [0.5, 1.0], 1e-3, 100.0, tol=1e-6, maxit=1, maxsweep=1)
    assert it == 2 and st & lg.LAGP_STATUS_MLE_MAXIT


def test_prescale_matches_numpy(lg):
    import torch

    rng = np.random.default_rng(720)
    X = rng.random((1000, 5))
    theta = np.array([0.2, 1.5, 7.0, 100.0, 0.03])
    out = torch.empty((1000, 5), dtype=torch.float64, device="cuda")
    lg.lagp_prescale(torch.from_numpy(X).cuda(), theta, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), X / np.sqrt(theta))


def test_local_mle_on_prescaled_inputs(lg):
    """Exhaustive and ray (p rays) search with two-stage local MLE on inputs
    scaled by global lengthscales: designs, estimates and predictions as the
    oracle's on numpy's scaled arrays."""
    import torch

    w = W.aniso8d(M=12, N=60_000)
    theta = np.array([0.2, 4.0, 50.0, 0.9, 100.0, 100.0, 100.0, 100.0])
    Xs = torch.empty((w.X.shape[0], 8), dtype=torch.float64, device="cuda")
    XXs = torch.empty((w.XX.shape[0], 8), dtype=torch.float64, device="cuda")
    lg.lagp_prescale(torch.from_numpy(w.X).cuda(), theta, Xs)
    lg.lagp_prescale(torch.from_numpy(w.XX).cuda(), theta, XXs)
    torch.cuda.synchronize()
    Xn, XXn = w.X / np.sqrt(theta), w.XX / np.sqrt(theta)
    assert np.array_equal(Xs.cpu().numpy(), Xn) and np.array_equal(XXs.cpu().numpy(), XXn)
    d = lg.Design(Xs, torch.from_numpy(w.y).cuda())
    try:
        for search, nr in ((W.SEARCH_EXHAUSTIVE, 0), (W.SEARCH_RAY, 8)):
            prm = w.params.replace(d=(1.0,), search=search, numrays=nr,
                                   scoring=W.SCORING_CHOL if search == W.SEARCH_EXHAUSTIVE else W.SCORING_PARTINV)
            out = d.predict_mle(XXs, prm, 2)
            torch.cuda.synchronize()
            g = {k: v.cpu().numpy() for k, v in out.items()}
            o = oracle.predict_mle(Xn, w.y, XXn, prm, 2)
            for k in ("sel", "dhat", "iters", "status", "mean", "s2"):
                assert np.array_equal(g[k], o[k]), (search, k)
    finally:
        d.close()


def test_sepfit_and_prescale_reject(lg):
    import torch

    XS = torch.zeros((4, 2), dtype=torch.float64, device="cuda")
    yS = torch.zeros(4, dtype=torch.float64, device="cuda")
    for args in ((1.0, 1e-3, 1e-3), (1.0, 1.0, 0.5), (-1.0, 1e-3, 10.0)):
        with pytest.raises(lg.LagpError) as e:
            lg.lagp_fit_separable(XS, yS, 1e-6, args[0], args[1], args[2])
        assert e.value.code == lg.LAGP_EINVAL
    big = torch.zeros((1025, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(lg.LagpError):
        lg.lagp_fit_separable(big, torch.zeros(1025, dtype=torch.float64, device="cuda"), 1e-6, 1.0, 1e-3, 10.0)
    with pytest.raises(lg.LagpError):
        lg.lagp_prescale(XS, np.array([1.0, 0.0]), XS)
    empty = torch.zeros((0, 2), dtype=torch.float64, device="cuda")
    assert lg.lagp_prescale(empty, np.array([1.0, 2.0]), empty) == 0
