"""HIP path vs the CPU oracle, through the C ABI (MI355X only)."""
import numpy as np
import pytest

import oracle
from paper_1409_0074_amd import workloads as W
from tests.parity import check_exact, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lg():
    import torch

    import paper_1409_0074_amd as lg

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lg.lib()  # loud failure when the HIP library is missing
    return lg


def _cands(lg, X, y, XX, ncand):
    import torch

    d = lg.Design(torch.from_numpy(X), torch.from_numpy(y))
    try:
        idx, d2 = d.candidates(torch.from_numpy(XX), ncand)
        torch.cuda.synchronize()
        return idx.cpu().numpy(), d2.cpu().numpy()
    finally:
        d.close()


# ------------------------------------------------------------------- kNN --

@pytest.mark.parametrize("case", ["uniform2d", "uniform8d", "grid_ties", "ragged", "p5", "p13", "offset3",
                                  "offset15", "offset18", "offset1e4"])
def test_candidates_bit_exact(lg, case):
    """offset3: coordinates in [3, 4]^4, the FP32 screen with norms far from
    zero; offset15: the FP32 screen with its slack at about 3/4 of the 5% of
    the estimated threshold it may take (the least margin for a wrong
    rounding bound); offset18 just past that limit and offset1e4 far past it
    ([1e4, 1e4 + 1]^4), where the FP64 screen runs instead."""
    rng = np.random.default_rng(101)
    if case == "uniform2d":
        w = W.tiny_2d()
        X, XX, nc = w.X, w.XX, 500
    elif case == "uniform8d":
        X, XX, nc = rng.random((30000, 8)), rng.random((24, 8)), 1000
    elif case == "grid_ties":
        X = W.grid2(120)
        XX = np.concatenate([X[[0, 7, 7000, 14399]], rng.random((5, 2))])  # grid points: many equal distances
        nc = 333
    elif case == "ragged":
        X, XX, nc = rng.random((1237, 3)), rng.random((13, 3)), 37
    elif case == "p5":
        X, XX, nc = rng.random((5000, 5)), rng.random((9, 5)), 64
    elif case.startswith("offset"):
        off = float(case[len("offset"):])
        X, XX, nc = rng.random((20000, 4)) + off, rng.random((11, 4)) + off, 200
    else:
        X, XX, nc = rng.random((3000, 13)), rng.random((3, 13)), 1
    gi, gd = _cands(lg, X, np.zeros(len(X)), XX, nc)
    oi, od = oracle.knn(X, XX, nc)
    assert np.array_equal(gi.astype(np.int64), oi)
    assert np.array_equal(gd, od)


@pytest.mark.parametrize("p", [1, 6, 7, 12, 16])
def test_candidates_every_chunk_count(lg, p):
    """The FP32 screen's product runs over ceil(p/4) K-chunks of coordinates
    (the row norm and the threshold enter as its start value): dimensions
    with one to four chunks, padded (p = 1, 6, 7) and whole (12, 16)."""
    rng = np.random.default_rng(150 + p)
    X, XX = rng.random((6000, p)), rng.random((70, p))  # 70 locations: two groups of 64, one ragged
    nc = 300
    idx, d2 = _cands(lg, X, X[:, 0].copy(), XX, nc)
    oi, od = oracle.knn(X, XX, nc)
    assert np.array_equal(idx.astype(np.int64), oi)
    assert np.array_equal(d2, od)


@pytest.mark.parametrize("case", ["uniform8d", "grid_ties"])
def test_candidates_forced_fallback_bit_exact(lg, case, monkeypatch):
    """The exact fallback scan (taken when the sampled threshold catches too
    few or too many rows) forced for every location."""
    monkeypatch.setenv("LAGP_KNN_FORCE_FALLBACK", "1")
    rng = np.random.default_rng(109)
    if case == "uniform8d":
        X, XX, nc = rng.random((20000, 8)), rng.random((10, 8)), 1000
    else:
        X = W.grid2(150)
        XX, nc = np.concatenate([X[[3, 11000]], rng.random((3, 2))]), 400
    gi, gd = _cands(lg, X, np.zeros(len(X)), XX, nc)
    oi, od = oracle.knn(X, XX, nc)
    assert np.array_equal(gi.astype(np.int64), oi) and np.array_equal(gd, od)


def test_candidates_large_design_bit_exact(lg):
    """The full-size 8-d design (N = 1e6) on a sample of locations."""
    w = W.uniform8d(M=12)
    gi, gd = _cands(lg, w.X, w.y, w.XX, 1000)
    oi, od = oracle.knn(w.X, w.XX, 1000)
    assert np.array_equal(gi.astype(np.int64), oi) and np.array_equal(gd, od)


@pytest.mark.parametrize("case", ["uniform8d_64", "sec51_55", "uniform8d_1"])
def test_candidates_short_lists(lg, case):
    """Short lists (the ray starts' candidates when rays snap over the whole
    design) sample a reduced share of the design for their threshold and
    collect more rows than they keep: still the exact lists, grid ties
    included."""
    if case == "sec51_55":
        w = W.paper2d(M=40)
        X, XX, nc = w.X, w.XX[::4], 55
    else:
        w = W.uniform8d(M=12)
        X, XX, nc = w.X, w.XX, int(case.split("_")[1])
    gi, gd = _cands(lg, X, np.zeros(len(X)), XX, nc)
    oi, od = oracle.knn(X, XX, nc)
    assert np.array_equal(gi.astype(np.int64), oi) and np.array_equal(gd, od)


def test_candidates_edge_sizes(lg):
    """ncand = N returns every row, in (d2, row) order."""
    rng = np.random.default_rng(102)
    X = rng.random((700, 2))
    x = rng.random((1, 2))
    gi, gd = _cands(lg, X, np.zeros(700), x, 700)
    oi, od = oracle.knn(X, x, 700)
    assert np.array_equal(gi.astype(np.int64), oi) and np.array_equal(gd, od)
    assert sorted(gi[0].tolist()) == list(range(700))


# ------------------------------------------------------- local designs ---

def test_exhaustive_uniform2d(lg):
    w = W.tiny_2d()
    g = run_gpu(w, w.params)
    assert np.all(g["status"] == 0)
    check_exact(w, w.params, g)


@pytest.mark.parametrize("case", ["uniform2d", "uniform8d", "grid"])
def test_exhaustive_free_run_bit_exact(lg, case):
    """FP64 exhaustive scoring sums every term in the defined order: the GPU's
    local designs, criterion values and predictions equal the oracle's bit for
    bit without replay."""
    rng = np.random.default_rng(108)
    if case == "uniform2d":
        w = W.tiny_2d()
    elif case == "uniform8d":
        X = rng.random((50000, 8))
        w = W.Workload("u8", X, W.f_sines8(X), rng.random((16, 8)),
                       W.Params(n0=6, n=50, ncand=1000, d=(0.5,) * 8, g=1e-6))
    else:
        X = W.grid2(200)
        w = W.Workload("grid", X, W.f_bump2(X), rng.random((10, 2)), W.Params(n0=6, n=80, ncand=700, d=(0.05,), g=1e-6))
    g = run_gpu(w, w.params)
    o = oracle.predict(w.X, w.y, w.XX, w.params)
    assert np.array_equal(g["sel"], o["sel"])
    assert np.array_equal(g["mean"], o["mean"]) and np.array_equal(g["s2"], o["s2"])
    assert np.array_equal(g["diag"][:, :, 0], o["diag"][:, :, 1])  # best ALC per step
    assert np.array_equal(g["diag"][:, :, 1], o["diag"][:, :, 2])  # runner-up


@pytest.mark.parametrize("sep", [True, False])
def test_exhaustive_uniform8d(lg, sep):
    rng = np.random.default_rng(103)
    X = rng.random((60000, 8))
    w = W.Workload("u8", X, W.f_sines8(X), rng.random((20, 8)),
                   W.Params(n0=6, n=50, ncand=1000, d=(0.5,) * 8 if sep else (0.5,), g=1e-6))
    g = run_gpu(w, w.params)
    check_exact(w, w.params, g)


@pytest.mark.parametrize("n,ncand,g_nug", [(64, 200, 1e-6), (100, 900, 1e-6), (70, 333, 1e-3)])
def test_exhaustive_large_n(lg, n, ncand, g_nug):
    """Local designs beyond 64 points take the 128-row tile path."""
    rng = np.random.default_rng(104)
    X = rng.random((20000, 2))
    w = W.Workload("u2", X, W.f_bump2(X), rng.random((6, 2)), W.Params(n0=6, n=n, ncand=ncand, d=(0.05,), g=g_nug))
    g = run_gpu(w, w.params)
    check_exact(w, w.params, g)


def test_exhaustive_grid_design(lg):
    """Grid designs tie in distance; the 2-d grid workload's shape, smaller."""
    X = W.grid2(300)
    rng = np.random.default_rng(105)
    w = W.Workload("grid", X, W.f_bump2(X), rng.random((8, 2)), W.Params(n0=6, n=60, ncand=800, d=(0.05,), g=1e-6))
    g = run_gpu(w, w.params)
    check_exact(w, w.params, g)


@pytest.mark.parametrize("R", [2, 10])
def test_ray_bit_exact(lg, R):
    """Every step of the ray search uses defined arithmetic on both sides:
    the GPU's designs and predictions equal the oracle's bit for bit."""
    if R == 2:
        w = W.tiny_2d(M=40)
        prm = w.params.replace(search=W.SEARCH_RAY, numrays=2)
    else:
        rng = np.random.default_rng(106)
        X = rng.random((40000, 8))
        w = W.Workload("u8", X, W.f_sines8(X), rng.random((12, 8)),
                       W.Params(n0=6, n=50, ncand=1000, search=W.SEARCH_RAY, numrays=10, d=(0.5,) * 8, g=1e-6))
        prm = w.params
    g = run_gpu(w, prm)
    o = oracle.predict(w.X, w.y, w.XX, prm)
    assert np.array_equal(g["sel"], o["sel"])
    assert np.array_equal(g["mean"], o["mean"]) and np.array_equal(g["s2"], o["s2"])
    assert np.array_equal(g["status"], o["status"])


def test_nn_mode_bit_exact(lg):
    w = W.tiny_2d(M=30)
    prm = w.params.replace(search=W.SEARCH_NN)
    g = run_gpu(w, prm, diag=False)
    o = oracle.predict(w.X, w.y, w.XX, prm)
    assert np.array_equal(g["sel"], o["sel"])
    assert np.array_equal(g["mean"], o["mean"]) and np.array_equal(g["s2"], o["s2"])


@pytest.mark.parametrize("M", [1, 7, 9])
def test_ragged_location_counts(lg, M):
    w = W.tiny_2d(M=M)
    g = run_gpu(w, w.params)
    check_exact(w, w.params, g)


def test_no_greedy_steps(lg):
    """n0 = n: the start is the whole design (no search)."""
    w = W.tiny_2d(M=5)
    prm = w.params.replace(n0=12, n=12)
    g = run_gpu(w, prm, diag=False)
    o = oracle.predict(w.X, w.y, w.XX, prm)
    assert np.array_equal(g["sel"], o["sel"]) and np.array_equal(g["mean"], o["mean"])


def test_empty_request(lg):
    import torch

    w = W.tiny_2d(M=1)
    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    out = d.predict(torch.zeros((0, 2), dtype=torch.float64), w.params)
    torch.cuda.synchronize()
    assert out["mean"].numel() == 0
    d.close()


def test_singular_start_status(lg):
    """Duplicates and g = 0: NaN and the NOTPD bit, as in the oracle."""
    X = np.repeat(np.random.default_rng(107).random((300, 2)), 2, axis=0)
    w = W.Workload("dup", X, W.f_bump2(X), X[:4].copy(), W.Params(n0=4, n=10, ncand=40, d=(0.1,), g=0.0))
    g = run_gpu(w, w.params)
    o = oracle.predict(w.X, w.y, w.XX, w.params)
    assert np.all(np.isnan(g["mean"])) and np.all(g["status"] & lg.LAGP_STATUS_NOTPD)
    assert np.array_equal(g["sel"], o["sel"])


def test_invalid_arguments_rejected(lg):
    import torch

    w = W.tiny_2d(M=2)
    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    bad = [dict(n=0), dict(n0=0), dict(ncand=10), dict(ncand=5000), dict(d=(-1.0,)), dict(g=-1.0),
           dict(search=W.SEARCH_RAY, numrays=40), dict(search=W.SEARCH_RAY, numrays=10, ncand=55), dict(search=7)]
    XX = torch.from_numpy(w.XX).cuda()
    out = [torch.empty(2, dtype=torch.float64, device="cuda") for _ in range(3)]
    for kw in bad:
        with pytest.raises(lg.LagpError) as e:
            lg.lagp_predict(d.handle, XX, lg.make_params(w.params.replace(**kw)), *out)
        assert e.value.code == lg.LAGP_EINVAL, kw
    d.close()
