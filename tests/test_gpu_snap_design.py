"""Ray search that snaps over the whole design (Sec. 5: ray searches are not
restricted to the N' nearest candidates) against the oracle, bit for bit
(MI355X only).

The oracle's reading of such a search is the same search with every design
row a candidate (its candidate list is then the whole design, nearest
first); the library keeps only the ray starts' candidates and finds each
snap target in the design's cell grid.  Designs, criterion values, means,
scales and status words must agree exactly."""
import numpy as np
import pytest

import oracle
from paper_1409_0074_amd import workloads as W

pytestmark = pytest.mark.gpu

FULL = W.SNAP_DESIGN


@pytest.fixture(scope="module")
def lg():
    import torch

    import paper_1409_0074_amd as lg

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lg.lib()
    return lg


def _need(n, n0, R):
    """Candidates the ray starts need: n - 1 + R + the largest round-robin
    offset t mod floor(sqrt t), t = 1 .. n - n0."""
    off = 0
    for t in range(1, n - n0 + 1):
        r = int(np.floor(np.sqrt(t)))
        off = max(off, t % r if r else 0)
    return n - 1 + R + off


def _uniform(seed, N, p, M, **kw):
    rng = np.random.default_rng(seed)
    X = rng.random((N, p))
    y = np.sin(3.0 * X).sum(axis=1) + X[:, 0] * X[:, -1]
    return W.Workload(f"u{p}", X, y, rng.random((M, p)), W.Params(**kw))


def _run(lg, w, prm, counts=False):
    import torch

    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    try:
        out = d.predict(torch.from_numpy(w.XX), prm, counts=counts)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    finally:
        d.close()


def _same(g, o, what):
    assert np.array_equal(g["sel"], o["sel"]), f"{what}: designs differ at {np.argwhere(g['sel'] != o['sel'])[:3]}"
    assert np.array_equal(g["mean"], o["mean"], equal_nan=True), what
    assert np.array_equal(g["s2"], o["s2"], equal_nan=True), what
    assert np.array_equal(g["status"], o["status"]), what
    assert np.array_equal(g["diag"][:, :, 0], o["diag"][:, :, 1]), what
    assert np.array_equal(g["diag"][:, :, 1], o["diag"][:, :, 2]), what


def _outside(g, w, prm):
    """How many chosen rows lie outside each location's ncand nearest."""
    idx, _ = oracle.knn(w.X, w.XX, prm.ncand)
    return sum(int(np.sum(~np.isin(g["sel"][m], idx[m]))) for m in range(w.XX.shape[0]))


def test_sec51_grid_one_ray(lg):
    """The Sec. 5.1 design (201 x 201 grid on [-2, 2]^2, f = -w(x1) w(x2)),
    one ray per step, n = 50: the candidate list holds only the starts'
    ranks, every snap goes to the grid."""
    w = W.paper2d(M=12, n=50, search=W.SEARCH_RAY, numrays=1)
    prm = w.params.replace(ncand=_need(50, 6, 1), snap=FULL)
    g = _run(lg, w, prm)
    _same(g, oracle.predict(w.X, w.y, w.XX, prm), "sec51 R=1")
    out = _outside(g, w, prm)
    print(f"rows outside the {prm.ncand} nearest: {out} of {g['sel'].size}")
    assert out > 0  # the snaps reach rows that are not candidates


def test_equidistant_rows_go_to_the_lower_rank(lg):
    """On the Sec. 5.1 grid a snap target can lie exactly midway between two
    grid rows (here at location 5, greedy step 146, d = 0.29907839...): the
    row of lower rank in the whole design's candidate order (nearer to x,
    then the lower row) is taken, as by a candidate list of the whole
    design."""
    w = W.paper2d(M=6, n=200, search=W.SEARCH_RAY, numrays=1)
    prm = w.params.replace(ncand=W.ray_candidates_needed(200, 6, 1), snap=FULL, d=(0.2990783938635783,))
    w = W.Workload(w.name, w.X, w.y, w.XX[5:6], prm)
    g = _run(lg, w, prm)
    o = oracle.predict(w.X, w.y, w.XX, prm)
    _same(g, o, "grid tie")
    assert o["diag"][0, 146, 4] == 0.0  # (the oracle's gap there: the two rows tie)


@pytest.mark.parametrize("p,R,n,N", [
    (1, 1, 30, 3000),    # a one-coordinate grid
    (2, 2, 90, 6000),    # design rows past 64 (the wider local plan)
    (3, 3, 40, 5000),    # three grid coordinates
    (4, 4, 40, 8000),    # the served workload's dimension
    (5, 5, 40, 6000),    # the generic-dimension kernel
    (8, 10, 50, 12000),  # the benchmark's ray shape: every ray of a step on one wave
    (12, 12, 40, 8000),  # more coordinates than the grid cuts
])
def test_shapes(lg, p, R, n, N):
    w = _uniform(900 + p + n, N, p, 6, n0=6, n=n, search=W.SEARCH_RAY, numrays=R, d=(0.1 * p,), g=1e-6)
    prm = w.params.replace(ncand=_need(n, 6, R) + 5, snap=FULL)
    g = _run(lg, w, prm)
    _same(g, oracle.predict(w.X, w.y, w.XX, prm), f"p={p} R={R} n={n}")


@pytest.mark.parametrize("p,R,n,N,ncand", [
    (8, 10, 50, 20000, 1000),  # the benchmark's shape: most snaps settled by the candidate list
    (2, 2, 40, 6000, 600),     # a dense 2-d design
    (4, 4, 60, 10000, 300),    # a shorter list: more snaps fall through to the grid
])
def test_long_lists_settle_snaps_exactly(lg, p, R, n, N, ncand):
    """With a long candidate list most snap targets lie so close to x that no
    row outside the list can be nearer than the best candidate; those snaps
    are settled by the list, the others by the grid: the same designs and
    predictions as the oracle's search over the whole design."""
    w = _uniform(940 + p, N, p, 6, n0=6, n=n, search=W.SEARCH_RAY, numrays=R, d=(0.1 * p,), g=1e-6)
    prm = w.params.replace(ncand=ncand, snap=FULL)
    g = _run(lg, w, prm)
    _same(g, oracle.predict(w.X, w.y, w.XX, prm), f"p={p} ncand={ncand}")


def test_four_wave_form(lg, monkeypatch):
    """LAGP_RAY_FORCE_WAVES=1 keeps the four-wave ray form: the same results."""
    monkeypatch.setenv("LAGP_RAY_FORCE_WAVES", "1")
    w = _uniform(931, 12000, 8, 6, n0=6, n=50, search=W.SEARCH_RAY, numrays=10, d=(0.8,), g=1e-6)
    prm = w.params.replace(ncand=_need(50, 6, 10), snap=FULL)
    _same(_run(lg, w, prm), oracle.predict(w.X, w.y, w.XX, prm), "four-wave form")


def test_whole_list_equals_candidate_snap(lg):
    """With the whole design as the candidate list both scopes are the same
    search: equal to each other and to the oracle."""
    w = _uniform(932, 3000, 2, 8, n0=6, n=40, search=W.SEARCH_RAY, numrays=2, d=(0.05,), g=1e-6)
    prm = w.params.replace(ncand=3000)
    g_c = _run(lg, w, prm)
    g_f = _run(lg, w, prm.replace(snap=FULL))
    for k in ("sel", "mean", "s2", "status", "diag"):
        assert np.array_equal(g_c[k], g_f[k], equal_nan=True), k
    _same(g_f, oracle.predict(w.X, w.y, w.XX, prm), "ncand = N")


def test_distinct_lengthscales_and_counts(lg):
    d4 = (0.2, 0.5, 1.0, 2.0)
    w = _uniform(933, 10000, 4, 6, n0=6, n=40, search=W.SEARCH_RAY, numrays=4, d=d4, g=1e-6)
    prm = w.params.replace(ncand=_need(40, 6, 4), snap=FULL)
    g = _run(lg, w, prm, counts=True)
    o = oracle.predict(w.X, w.y, w.XX, prm)
    _same(g, o, "distinct d_k")
    assert np.array_equal(g["counts"][:, :, 0], o["diag"][:, :, 5].astype(np.int32))


def test_constant_coordinate_and_duplicates(lg):
    """A coordinate that never varies (one cell along it) and every row
    duplicated (equal distances: the lower row wins)."""
    rng = np.random.default_rng(934)
    X = rng.random((2500, 3))
    X[:, 1] = 0.5
    X = np.repeat(X, 2, axis=0)
    y = np.sin(4.0 * X[:, 0]) + X[:, 2]
    XX = rng.random((6, 3))
    XX[:, 1] = 0.5
    w = W.Workload("dup3", X, y, XX, W.Params(n0=6, n=30, search=W.SEARCH_RAY, numrays=3, d=(0.3,), g=1e-4))
    prm = w.params.replace(ncand=_need(30, 6, 3) + 10, snap=FULL)
    _same(_run(lg, w, prm), oracle.predict(w.X, w.y, w.XX, prm), "duplicates")


def test_local_mle_with_design_snap(lg):
    """Two-stage local MLE over ray searches that snap over the design."""
    import torch

    w = _uniform(935, 8000, 2, 5, n0=6, n=30, search=W.SEARCH_RAY, numrays=2, d=(0.05,), g=1e-6)
    prm = w.params.replace(ncand=_need(30, 6, 2), snap=FULL)
    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    try:
        g = d.predict_mle(torch.from_numpy(w.XX), prm, mode=2)
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in g.items() if v is not None}
    finally:
        d.close()
    o = oracle.predict_mle(w.X, w.y, w.XX, prm, mode=2)
    for k in ("sel", "mean", "s2", "dhat", "status"):
        assert np.array_equal(g[k], o[k], equal_nan=True), k


def test_scope_is_checked(lg):
    import torch

    w = _uniform(936, 2000, 2, 2, n0=6, n=20, d=(0.1,), g=1e-6)
    d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
    try:
        with pytest.raises(lg.LagpError):  # exhaustive search has no snap
            d.predict(torch.from_numpy(w.XX), w.params.replace(ncand=200, snap=FULL))
        with pytest.raises(lg.LagpError):
            d.predict(torch.from_numpy(w.XX), w.params.replace(ncand=200, search=W.SEARCH_RAY, numrays=2, snap=7))
    finally:
        d.close()
