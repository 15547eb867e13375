"""Mixed precision form (FP32 MFMA screen with certified error bounds, the
shortlist it cannot rule out re-scored exactly in FP64) against the oracle's
FP64 run.  MI355X only.

The screen bounds every candidate's FP64 criterion from above and below;
every candidate whose upper bound reaches the second largest lower bound is
re-scored by the FP64 scoring itself, so the FP64 argmax and runner-up are
always among the re-scored values: designs, per-step criterion values,
means, scales and status words equal the oracle's FP64 run bit for bit, at
any conditioning.  How much of the candidate set the certificate has to
re-score (the form's cost) is reported, not asserted."""
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


def _run(lg, w, prm):
    import torch

    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    try:
        out = d.predict(torch.from_numpy(w.XX), prm, counts=True)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    finally:
        d.close()


def _equal_to_oracle(g, o, what):
    assert np.array_equal(g["sel"], o["sel"]), f"{what}: designs differ at {np.argwhere(g['sel'] != o['sel'])[:3]}"
    assert np.array_equal(g["mean"], o["mean"], equal_nan=True), what
    assert np.array_equal(g["s2"], o["s2"], equal_nan=True), what
    assert np.array_equal(g["status"], o["status"]), what
    assert np.array_equal(g["diag"][:, :, 0], o["diag"][:, :, 1]), what  # best criterion per step
    assert np.array_equal(g["diag"][:, :, 1], o["diag"][:, :, 2]), what  # runner-up


def _report(g, prm, what):
    ct = g["counts"]
    free = prm.ncand - (prm.n0 + np.arange(prm.n - prm.n0))
    frac = ct[:, :, 0] / free[None, :]
    tiles = ct[:, :, 1] / ((prm.ncand + 15) // 16)
    print(f"{what}: shortlist mean {ct[:, :, 0].mean():.1f} max {ct[:, :, 0].max()} candidates "
          f"({frac.mean():.3f} of the free ones); tiles re-scored {tiles.mean():.3f} of all")
    assert np.all(ct[:, :, 0] >= 1) and np.all(ct[:, :, 0] <= free[None, :])
    return frac.mean()


def test_mixed_equals_fp64_on_the_grid_workload_shape(lg):
    """The 1000 x 1000 grid, N' = 4000, n = 100, d = 0.05, g = 1e-6 (cond(K_J)
    up to ~1e8, where FP32 cannot resolve (1+g) - k^T K^{-1} k: the bounds
    widen the shortlist accordingly), 32 locations: equal to the oracle's
    FP64 run bit for bit."""
    w = W.grid2d(M=32, precision=W.PREC_MIXED)
    g = _run(lg, w, w.params)
    o = oracle.predict(w.X, w.y, w.XX, w.params.replace(precision=W.PREC_FP64))
    _equal_to_oracle(g, o, "grid2d mixed")
    _report(g, w.params, "grid2d mixed")


def test_mixed_equals_fp64_when_well_conditioned(lg):
    """8-d uniform design, d = 0.5 per dimension (the benchmark's local shape)."""
    rng = np.random.default_rng(301)
    X = rng.random((60000, 8))
    prm = W.Params(n0=6, n=50, ncand=1000, d=(0.5,) * 8, g=1e-6, precision=W.PREC_MIXED)
    w = W.Workload("u8", X, W.f_sines8(X), rng.random((24, 8)), prm)
    g = _run(lg, w, prm)
    o = oracle.predict(w.X, w.y, w.XX, prm.replace(precision=W.PREC_FP64))
    _equal_to_oracle(g, o, "uniform8d mixed")
    _report(g, prm, "uniform8d mixed")


@pytest.mark.parametrize("g_nug,d", [(1e-2, 0.1), (1e-4, 0.1), (1e-6, 0.1), (0.0, 0.02)])
def test_mixed_equals_fp64_across_conditioning(lg, g_nug, d):
    """From a large nugget (the bounds separate the winner from most
    candidates) to none at all (g = 0: v may reach 0 and the VNONPOS flag
    must be reproduced)."""
    w = W.tiny_2d(M=12)
    prm = w.params.replace(precision=W.PREC_MIXED, g=g_nug, d=(d,))
    g = _run(lg, w, prm)
    o = oracle.predict(w.X, w.y, w.XX, prm.replace(precision=W.PREC_FP64))
    _equal_to_oracle(g, o, f"tiny 2-d mixed g={g_nug} d={d}")
    _report(g, prm, f"tiny 2-d mixed g={g_nug} d={d}")


@pytest.mark.parametrize("n,ncand", [(64, 300), (100, 900), (128, 4096)])
def test_mixed_equals_fp64_large_designs(lg, n, ncand):
    """Local designs past 64 points (the 128-row tiles), up to the largest n
    and N'."""
    rng = np.random.default_rng(303)
    X = rng.random((30000, 2))
    prm = W.Params(n0=6, n=n, ncand=ncand, d=(0.05,), g=1e-6, precision=W.PREC_MIXED)
    w = W.Workload("u2", X, W.f_bump2(X), rng.random((4, 2)), prm)
    g = _run(lg, w, prm)
    o = oracle.predict(w.X, w.y, w.XX, prm.replace(precision=W.PREC_FP64))
    _equal_to_oracle(g, o, f"mixed n={n} ncand={ncand}")
    _report(g, prm, f"mixed n={n} ncand={ncand}")


def test_counts_of_the_fp64_and_ray_forms(lg):
    """The FP64 forms report every free candidate scored; the ray form's
    per-step Brent evaluations equal the oracle's (the same iterations)."""
    w = W.tiny_2d(M=10)
    for scoring in (W.SCORING_PARTINV, W.SCORING_CHOL):
        prm = w.params.replace(scoring=scoring)
        g = _run(lg, w, prm)
        free = prm.ncand - (prm.n0 + np.arange(prm.n - prm.n0))
        assert np.array_equal(g["counts"][:, :, 0], np.broadcast_to(free, g["counts"].shape[:2]))
        assert np.all(g["counts"][:, :, 1] == 0)
    prm = w.params.replace(search=W.SEARCH_RAY, numrays=3)
    g = _run(lg, w, prm)
    o = oracle.predict(w.X, w.y, w.XX, prm)
    assert np.array_equal(g["sel"], o["sel"])
    assert np.array_equal(g["counts"][:, :, 0], o["diag"][:, :, 5].astype(np.int32))
    assert np.all(g["counts"][:, :, 1] <= g["counts"][:, :, 0]) and np.all(g["counts"][:, :, 1] >= 1)
    print(f"ray R=3: evaluations per step mean {g['counts'][:, :, 0].mean():.1f}, per ray mean "
          f"{g['counts'][:, :, 0].mean() / 3:.1f}, most on one ray {g['counts'][:, :, 1].max()}")
