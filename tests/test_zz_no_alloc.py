"""lagp_predict_noalloc (the entry point that allocates nothing: its
workspace is a fixed per-device scratch array) against lagp_predict, through
the C ABI (MI355X only).  Both run the same kernels, so designs, criterion
values, predictions and status words must be equal bit for bit.  Each case
makes two calls in a row, the second with a smaller input, so the second
runs on the scratch contents the first left behind; the larger calls span
several chunks of the scratch."""
import numpy as np
import pytest

from paper_1409_0074_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1409_0074_amd as lg

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lg.lib()
    rng = np.random.default_rng(601)
    X = rng.random((120_000, 8))
    d = lg.Design(torch.from_numpy(X), torch.from_numpy(W.f_sines8(X)))
    yield lg, d, rng
    d.close()


def _call(lg, d, fn, XX, prm):
    import torch

    P = lg.make_params(prm)
    M = XX.shape[0]
    n0 = prm.n if prm.search == W.SEARCH_NN else prm.n0
    dev = dict(dtype=torch.float64, device="cuda")
    out = dict(mean=torch.full((M,), 7.0, **dev), s2=torch.full((M,), 7.0, **dev), df=torch.full((M,), 7.0, **dev),
               sel=torch.full((M, prm.n), -7, dtype=torch.int32, device="cuda"),
               diag=torch.full((M, prm.n - n0, 2), 7.0, **dev),
               status=torch.full((M,), -7, dtype=torch.int32, device="cuda"))
    XXd = torch.from_numpy(XX).cuda()
    fn(d.handle, XXd, P, out["mean"], out["s2"], out["df"], out["sel"], out["diag"], out["status"])
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("case,M1,M2", [
    ("chol", 1700, 300),     # Cholesky scoring: about 1,150 locations per scratch chunk here
    ("chol_stream", 700, 60),  # n = 100: columns streamed from slots in the scratch, ~550 per chunk
    ("partinv", 260, 37),    # partitioned inverse: about 115 per chunk (kernel rows in the workspace)
    ("ray", 150, 20),
    ("ray_design", 150, 20),  # snap over the whole design: the design's grid is built beforehand
    ("mixed", 120, 9),
])
def test_noalloc_equals_predict_twice(env, case, M1, M2):
    lg, d, rng = env
    prm = W.Params(n0=6, n=50, ncand=1000, d=(0.5,) * 8, g=1e-6)
    if case == "chol":
        prm = prm.replace(scoring=W.SCORING_CHOL)
    elif case == "chol_stream":
        prm = prm.replace(scoring=W.SCORING_CHOL, n=100)
    elif case == "ray":
        prm = prm.replace(search=W.SEARCH_RAY, numrays=8)
    elif case == "ray_design":
        prm = prm.replace(search=W.SEARCH_RAY, numrays=8, ncand=100, snap=W.SNAP_DESIGN)
        lg.lagp_design_build_grid(d.handle)
    elif case == "mixed":
        prm = prm.replace(precision=W.PREC_MIXED)
    for M in (M1, M2):
        XX = rng.random((M, 8))
        a = _call(lg, d, lg.lagp_predict_noalloc, XX, prm)
        b = _call(lg, d, lg.lagp_predict, XX, prm)
        for k in b:
            assert np.array_equal(a[k], b[k]), (case, M, k)
        assert np.all(a["status"] == 0) and np.all(a["df"] == prm.n)


def test_noalloc_rejects_what_the_scratch_cannot_hold():
    """A 2e7-row 4-d design with 64 candidates: the candidate search's
    per-call subsample alone (N/8 rows of 4 coordinates, 80 MB) exceeds the
    64 MiB scratch."""
    import torch

    import paper_1409_0074_amd as lg

    rng = np.random.default_rng(602)
    X = torch.from_numpy(rng.random((20_000_000, 4)))
    d = lg.Design(X, X[:, 0].clone())
    try:
        prm = W.Params(n0=4, n=10, ncand=64, d=(0.1,), g=1e-6, scoring=W.SCORING_CHOL)
        XX = torch.from_numpy(rng.random((4, 4))).cuda()
        out = [torch.empty(4, dtype=torch.float64, device="cuda") for _ in range(3)]
        with pytest.raises(lg.LagpError) as e:
            lg.lagp_predict_noalloc(d.handle, XX, lg.make_params(prm), *out)
        assert e.value.code == lg.LAGP_ENOMEM and "scratch" in str(e.value)
        # the allocating entry point runs the same request
        lg.lagp_predict(d.handle, XX, lg.make_params(prm), *out)
        torch.cuda.synchronize()
        assert np.all(np.isfinite(out[0].cpu().numpy()))
    finally:
        d.close()
