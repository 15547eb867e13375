"""Local MLE of the lengthscale and the two-stage re-design vs the oracle
(MI355X only).

The library's Newton iteration, its likelihood derivatives, the searches
under the estimates and the prediction use the oracle's arithmetic in the
oracle's order, so estimates, evaluation counts, designs, means, scales and
status words must be equal bit for bit.  The oracle's O8 is pinned to numpy
and scipy maximisers and to 40-digit arithmetic."""
import numpy as np
import pytest

import oracle
from paper_1409_0074_amd import workloads as W

pytestmark = pytest.mark.gpu

CHOL = W.SCORING_CHOL


@pytest.fixture(scope="module")
def lg():
    import torch

    import paper_1409_0074_amd as lg

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lg.lib()
    return lg


def _gpu(lg, w, prm, mode, **kw):
    import torch

    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    try:
        out = d.predict_mle(torch.from_numpy(w.XX), prm, mode, **kw)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        d.close()


def _exact(lg, w, prm, mode, **kw):
    g = _gpu(lg, w, prm, mode, **kw)
    o = oracle.predict_mle(w.X, w.y, w.XX, prm, mode, **kw)
    assert np.array_equal(g["sel"], o["sel"])
    assert np.array_equal(g["dhat"], o["dhat"])
    assert np.array_equal(g["iters"], o["iters"])
    assert np.array_equal(g["status"], o["status"])
    assert np.array_equal(g["mean"], o["mean"], equal_nan=True)
    assert np.array_equal(g["s2"], o["s2"], equal_nan=True)
    return g, o


@pytest.mark.parametrize("mode", [1, 2])
def test_mle_uniform2d(lg, mode):
    """N = 4000, p = 2, n = 50, N' = 500, d0 = 0.1."""
    w = W.tiny_2d(M=24)
    g, _ = _exact(lg, w, w.params.replace(scoring=CHOL), mode)
    assert np.all(g["status"] & ~(lg.LAGP_STATUS_MLE_BOUND) == 0)
    print(f"mode {mode}: dhat {np.round(g['dhat'][:6], 4)}, evaluations {g['iters'][:6]}")


@pytest.mark.parametrize("mode", [1, 2])
def test_mle_uniform8d(lg, mode):
    """p = 8, n = 50, N' = 1000, isotropic d0 = 0.5."""
    rng = np.random.default_rng(211)
    X = rng.random((60000, 8))
    w = W.Workload("u8", X, W.f_sines8(X), rng.random((12, 8)),
                   W.Params(n0=6, n=50, ncand=1000, d=(0.5,), g=1e-6, scoring=CHOL))
    _exact(lg, w, w.params, mode)


@pytest.mark.parametrize("search,numrays", [(W.SEARCH_RAY, 1), (W.SEARCH_RAY, 2), (W.SEARCH_NN, 0)])
@pytest.mark.parametrize("mode", [1, 2])
def test_mle_rays_and_nearest_neighbours(lg, search, numrays, mode):
    """The other two design searches under local inference (Sec. 5):
    rays (k_local's lockstep Brent searches under each location's own
    estimate at stage two) and the nearest-neighbour design."""
    w = W.tiny_2d(M=16)
    g, _ = _exact(lg, w, w.params.replace(search=search, numrays=numrays), mode)
    assert np.all(np.isfinite(g["mean"]))


@pytest.mark.parametrize("mode", [1, 2])
def test_mle_partitioned_inverse_scoring(lg, mode):
    """Exhaustive search scored by partitioned-inverse updates (k_local,
    any N' the kernel takes) under local inference."""
    w = W.tiny_2d(M=12)
    _exact(lg, w, w.params.replace(ncand=1200), mode)


def test_mle_rays_uniform8d(lg):
    """p = 8, n = 50, N' = 1000, 8 rays, two stages."""
    rng = np.random.default_rng(212)
    X = rng.random((60000, 8))
    w = W.Workload("u8r", X, W.f_sines8(X), rng.random((8, 8)),
                   W.Params(n0=6, n=50, ncand=1000, search=W.SEARCH_RAY, numrays=8, d=(0.5,), g=1e-6))
    _exact(lg, w, w.params, 2)


def test_mle_bounds_and_budget(lg):
    """A narrow range pins estimates to a bound; a tiny budget stops the
    iteration: both reported as the oracle reports them."""
    w = W.tiny_2d(M=10)
    prm = w.params.replace(scoring=CHOL)
    g, _ = _exact(lg, w, prm, 2, dmin=0.2, dmax=0.5)
    assert np.all(g["status"] & lg.LAGP_STATUS_MLE_BOUND)
    g, _ = _exact(lg, w, prm, 1, maxit=2)
    assert np.all(g["status"] & lg.LAGP_STATUS_MLE_MAXIT)


@pytest.mark.parametrize("p,n,n0,ncand", [(3, 20, 20, 64), (5, 33, 4, 333), (12, 40, 6, 300)])
def test_mle_shapes(lg, p, n, n0, ncand):
    w = W.small_case(300 + p + n, 5000, p, 7, n0=n0, n=n, ncand=ncand, d=(0.3 * p,), g=1e-5, scoring=CHOL)
    _exact(lg, w, w.params, 2)


@pytest.mark.parametrize("search", [W.SEARCH_EXHAUSTIVE, W.SEARCH_RAY])
def test_mle_singular_start(lg, search):
    """Duplicated points and g = 0: the first search fails; NaN, NOTPD and
    the lengthscale searched under, as in the oracle (the second stage
    skips those locations in both search kernels)."""
    X = np.repeat(np.random.default_rng(107).random((300, 2)), 2, axis=0)
    prm = W.Params(n0=4, n=10, ncand=40, d=(0.1,), g=0.0, search=search, numrays=2,
                   scoring=CHOL if search == W.SEARCH_EXHAUSTIVE else W.SCORING_PARTINV)
    w = W.Workload("dup", X, W.f_bump2(X), X[:4].copy(), prm)
    g, _ = _exact(lg, w, w.params, 2)
    assert np.all(np.isnan(g["mean"])) and np.all(g["status"] & lg.LAGP_STATUS_NOTPD)


def test_mle_with_given_candidates(lg):
    """Candidate lists from lagp_candidates give the same results as the
    entry point's own neighbour search."""
    import torch

    w = W.tiny_2d(M=9)
    prm = w.params.replace(scoring=CHOL)
    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    try:
        XX = torch.from_numpy(w.XX).cuda()
        idx, _ = d.candidates(XX, prm.ncand)
        M = XX.shape[0]
        f64 = dict(dtype=torch.float64, device="cuda")
        out = [torch.empty(M, **f64) for _ in range(4)]
        sel = torch.empty((M, prm.n), dtype=torch.int32, device="cuda")
        lg.lagp_predict_mle(d.handle, XX, idx, lg.make_params(prm), lg.make_mle_params(2), *out, sel)
        ref = d.predict_mle(XX, prm, 2)
        torch.cuda.synchronize()
        assert torch.equal(out[0], ref["mean"]) and torch.equal(out[3], ref["dhat"]) and torch.equal(sel, ref["sel"])
    finally:
        d.close()


def test_mle_rejects_unsupported(lg):
    import torch

    w = W.tiny_2d(M=2)
    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    XX = torch.from_numpy(w.XX).cuda()
    out = [torch.empty(2, dtype=torch.float64, device="cuda") for _ in range(4)]
    ok = w.params.replace(scoring=CHOL)
    bad = [(ok, lg.make_mle_params(3)), (ok.replace(d=(0.1, 0.2)), lg.make_mle_params(1)),
           (ok.replace(scoring=W.SCORING_PARTINV, precision=W.PREC_MIXED), lg.make_mle_params(1)),
           (ok, lg.make_mle_params(1, dmin=1.0, dmax=0.5)),
           (ok.replace(n=257, ncand=600), lg.make_mle_params(1))]
    for prm, q in bad:
        with pytest.raises(lg.LagpError) as e:
            lg.lagp_predict_mle(d.handle, XX, None, lg.make_params(prm), q, *out)
        assert e.value.code == lg.LAGP_EINVAL
    d.close()
