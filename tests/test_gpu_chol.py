"""Exhaustive search by incremental Cholesky columns vs the oracle's
Cholesky form (MI355X only).

Both sides grow the same factor in the same order (index-order fused
multiply-add sums, IEEE division and square root, the same exp), so the
GPU's designs, criterion values and predictions must equal the oracle's bit
for bit.  The oracle's Cholesky form is itself pinned to 40-digit arithmetic
and to the partitioned-inverse form where both are well conditioned."""
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
    assert np.array_equal(g["sel"], o["sel"])
    assert np.array_equal(g["mean"], o["mean"], equal_nan=True)
    assert np.array_equal(g["s2"], o["s2"], equal_nan=True)
    assert np.array_equal(g["status"], o["status"])
    if diag and prm.n > prm.n0:
        assert np.array_equal(g["diag"][:, :, 0], o["diag"][:, :, 1])  # best criterion per step
        assert np.array_equal(g["diag"][:, :, 1], o["diag"][:, :, 2])  # runner-up
    return g, o


def test_chol_uniform2d(lg):
    """N = 4000, p = 2, n = 50, N' = 500, all 100 locations."""
    w = W.tiny_2d()
    g, _ = _exact(w, w.params.replace(scoring=CHOL))
    assert np.all(g["status"] == 0) and np.all(g["df"] == w.params.n)


@pytest.mark.parametrize("sep", [True, False])
def test_chol_uniform8d(lg, sep):
    """p = 8, n = 50, N' = 1000 (the benchmark's local shape), separable and
    isotropic lengthscales."""
    rng = np.random.default_rng(111)
    X = rng.random((60000, 8))
    w = W.Workload("u8", X, W.f_sines8(X), rng.random((24, 8)),
                   W.Params(n0=6, n=50, ncand=1000, d=(0.5,) * 8 if sep else (0.5,), g=1e-6, scoring=CHOL))
    g, _ = _exact(w, w.params)
    assert np.all(g["status"] == 0)


@pytest.mark.parametrize("p,n,n0,ncand", [
    (1, 20, 3, 64),      # one dimension, a single wave
    (3, 32, 6, 77),      # ragged candidate count, the small register form at its limit
    (3, 33, 6, 333),     # the large form just past the small one
    (5, 50, 1, 1024),    # one starting point, the largest candidate set
    (12, 40, 6, 300),    # p > 8
    (16, 50, 6, 512),    # the largest p at its largest candidate set
    (2, 50, 50, 200),    # n0 = n: no greedy step
    (2, 24, 6, 24),      # N' = n: every candidate is taken
])
def test_chol_shapes(lg, p, n, n0, ncand):
    w = W.small_case(120 + p + n, 5000, p, 9, n0=n0, n=n, ncand=ncand, d=(0.3 * p,) * p, g=1e-5, scoring=CHOL)
    g, _ = _exact(w, w.params, diag=n0 < n)
    assert np.all(g["status"] == 0)


def test_chol_grid_ties(lg):
    """Grid design (distance ties in the candidate lists), n = 50, N' = 900."""
    X = W.grid2(300)
    rng = np.random.default_rng(112)
    w = W.Workload("grid", X, W.f_bump2(X), rng.random((12, 2)),
                   W.Params(n0=6, n=50, ncand=900, d=(0.05,), g=1e-6, scoring=CHOL))
    _exact(w, w.params)


def test_chol_agrees_with_partitioned_inverse_path_when_well_conditioned(lg):
    """With a large nugget both scoring forms are accurate, so the library's
    two exhaustive paths choose the same designs and agree to 1e-10."""
    w = W.tiny_2d(M=40)
    prm = w.params.replace(g=1e-2, n=40)
    g1 = run_gpu(w, prm)
    g2 = run_gpu(w, prm.replace(scoring=CHOL))
    assert np.array_equal(g1["sel"], g2["sel"])
    assert np.allclose(g2["mean"], g1["mean"], rtol=1e-10, atol=1e-14)
    assert np.allclose(g2["s2"], g1["s2"], rtol=1e-10, atol=0)


def test_chol_singular_start(lg):
    """Duplicated design points and g = 0: NaN and the NOTPD bit, the n0
    nearest reported, as in the oracle."""
    X = np.repeat(np.random.default_rng(107).random((300, 2)), 2, axis=0)
    w = W.Workload("dup", X, W.f_bump2(X), X[:4].copy(), W.Params(n0=4, n=10, ncand=40, d=(0.1,), g=0.0,
                                                                 scoring=CHOL))
    g, _ = _exact(w, w.params, diag=False)  # no greedy step runs
    assert np.all(np.isnan(g["mean"])) and np.all(g["status"] & lg.LAGP_STATUS_NOTPD)


@pytest.mark.parametrize("M", [1, 7, 65])
def test_chol_ragged_locations(lg, M):
    w = W.tiny_2d(M=M)
    _exact(w, w.params.replace(scoring=CHOL))


def test_chol_rejects_unsupported(lg):
    import torch

    w = W.tiny_2d(M=2)
    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    # (past the on-chip sizes the columns stream from a workspace: n = 51 or
    # ncand = 1025 are accepted; the limits are LAGP_MAX_N and LAGP_MAX_NCAND)
    bad = [dict(n=257), dict(ncand=4097, n=50), dict(search=W.SEARCH_RAY, numrays=2), dict(precision=W.PREC_MIXED),
           dict(search=W.SEARCH_NN)]
    XX = torch.from_numpy(w.XX).cuda()
    out = [torch.empty(2, dtype=torch.float64, device="cuda") for _ in range(3)]
    for kw in bad:
        with pytest.raises(lg.LagpError) as e:
            lg.lagp_predict(d.handle, XX, lg.make_params(w.params.replace(scoring=CHOL, **kw)), *out)
        assert e.value.code == lg.LAGP_EINVAL, kw
    with pytest.raises(lg.LagpError):
        lg.lagp_predict(d.handle, XX, lg.make_params(w.params.replace(scoring=2)), *out)
    d.close()
