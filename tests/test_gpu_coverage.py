"""HIP path vs the CPU oracle on the shapes the other parity tests leave
out (MI355X only): ray search in 1, 3, 4, 5 and 12 dimensions and with
local designs past 64 points, separable kernels with distinct lengthscales
per dimension under every search, and requests answered by the server.
Every comparison is against the oracle's own independent run, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1409_0074_amd import workloads as W
from tests.parity import run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lg():
    import torch

    import paper_1409_0074_amd as lg

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lg.lib()
    return lg


def _same(g, o, what=""):
    assert np.array_equal(g["sel"], o["sel"]), f"{what}: designs differ at {np.argwhere(g['sel'] != o['sel'])[:3]}"
    assert np.array_equal(g["mean"], o["mean"], equal_nan=True), what
    assert np.array_equal(g["s2"], o["s2"], equal_nan=True), what
    assert np.array_equal(g["status"], o["status"]), what


def _uniform(seed, N, p, M, **kw):
    rng = np.random.default_rng(seed)
    X = rng.random((N, p))
    y = np.sin(3.0 * X).sum(axis=1) + X[:, 0] * X[:, -1]
    return W.Workload(f"u{p}", X, y, rng.random((M, p)), W.Params(**kw))


# ------------------------------------------------------------ ray search --

@pytest.mark.parametrize("p,R,n,ncand", [
    (1, 1, 30, 200),    # the one-dimensional instantiation
    (3, 3, 40, 400),    # three dimensions
    (4, 4, 50, 1000),   # four dimensions, the served workload's ray shape at n = 50
    (5, 5, 40, 500),    # the generic-dimension instantiation
    (12, 12, 40, 600),  # generic, p > 8
    (4, 4, 100, 1000),  # the served workload's n = 100 rays: design rows past 64 on a second lane half
    (2, 3, 90, 700),    # two dimensions past 64 rows
])
def test_ray_shapes_bit_exact(lg, p, R, n, ncand):
    w = _uniform(500 + p + n, 8000 if p < 8 else 20000, p, 6, n0=6, n=n, ncand=ncand, search=W.SEARCH_RAY,
                 numrays=R, d=(0.1 * p,), g=1e-6)
    g = run_gpu(w, w.params)
    o = oracle.predict(w.X, w.y, w.XX, w.params)
    _same(g, o, f"rays p={p} R={R} n={n}")
    assert np.all(g["status"] == 0)


# ------------------------------------------- distinct lengthscales per dim --

D4 = (0.2, 0.5, 1.0, 2.0)


@pytest.mark.parametrize("form", ["partinv", "chol", "ray", "nn"])
def test_separable_distinct_lengthscales_bit_exact(lg, form):
    """d_k = 0.2, 0.5, 1, 2: a per-dimension indexing mistake (a swapped or
    shared d_k) changes the kernel values and so the designs."""
    kw = dict(n0=6, n=50, ncand=800, d=D4, g=1e-6)
    if form == "chol":
        kw["scoring"] = W.SCORING_CHOL
    elif form == "ray":
        kw.update(search=W.SEARCH_RAY, numrays=4)
    elif form == "nn":
        kw["search"] = W.SEARCH_NN
    w = _uniform(520, 30000, 4, 10, **kw)
    g = run_gpu(w, w.params, diag=form != "nn")
    o = oracle.predict(w.X, w.y, w.XX, w.params)
    _same(g, o, form)
    # the same inputs under the lengthscales in another order give other designs
    o2 = oracle.predict(w.X, w.y, w.XX, w.params.replace(d=D4[::-1]))
    assert not np.array_equal(o2["sel"], o["sel"]) or form == "nn"


def test_separable_distinct_lengthscales_eight_dims(lg):
    """Eight distinct d_k under the Cholesky form (the benchmark's scoring)
    and the partitioned-inverse form."""
    d8 = tuple(0.25 * (k + 1) for k in range(8))
    w = _uniform(521, 40000, 8, 8, n0=6, n=50, ncand=1000, d=d8, g=1e-6)
    for scoring in (W.SCORING_CHOL, W.SCORING_PARTINV):
        prm = w.params.replace(scoring=scoring)
        g = run_gpu(w, prm)
        _same(g, oracle.predict(w.X, w.y, w.XX, prm), f"scoring {scoring}")


def test_separable_distinct_lengthscales_mixed(lg):
    """The mixed form with distinct d_k on a well-conditioned design: its
    re-scored choices are the FP64 ones, so it equals the oracle's FP64 run."""
    w = _uniform(522, 30000, 4, 10, n0=6, n=40, ncand=600, d=D4, g=1e-4, precision=W.PREC_MIXED)
    g = run_gpu(w, w.params)
    o = oracle.predict(w.X, w.y, w.XX, w.params.replace(precision=W.PREC_FP64))
    _same(g, o, "mixed")


# --------------------------------------------------------------- serving --

def test_served_requests_equal_the_oracle(lg):
    """A mix of requests (exhaustive under both scoring forms, rays at
    n = 50 and 100, nearest neighbours, distinct d_k, the mixed form) through
    the server: every request's results equal the oracle's own run."""
    rng = np.random.default_rng(530)
    X = rng.random((60000, 4))
    y = W.f_mix4(X)
    base = W.Params(n0=6, n=50, ncand=1000, d=(0.1,), g=1e-6)
    prms = [
        base.replace(n=30, scoring=W.SCORING_CHOL),
        base.replace(scoring=W.SCORING_CHOL, d=D4),
        base.replace(n=100),
        base.replace(search=W.SEARCH_RAY, numrays=4),
        base.replace(n=100, search=W.SEARCH_RAY, numrays=4),
        base.replace(search=W.SEARCH_NN),
        base.replace(n=40, g=1e-4, precision=W.PREC_MIXED),
    ]
    reqs = [(rng.random((int(m), 4)), prm) for m, prm in zip([3, 17, 5, 9, 4, 11, 6], prms)]
    import torch

    d = lg.Design(torch.from_numpy(X), torch.from_numpy(y))
    srv = lg.lagp_server_create(d.handle, 4 << 30, 4)
    try:
        tickets = [lg.lagp_server_submit(srv, XX, lg.make_params(prm))[1] for XX, prm in reqs]
        res = [lg.lagp_server_fetch(srv, t, XX.shape[0], prm.n) for t, (XX, prm) in zip(tickets, reqs)]
    finally:
        lg.lagp_server_destroy(srv)
        d.close()
    for k, ((XX, prm), r) in enumerate(zip(reqs, res)):
        o = oracle.predict(X, y, XX, prm.replace(precision=W.PREC_FP64))
        _same(r, o, f"request {k}")


def test_merged_batch_of_varied_requests_equals_the_oracle(lg):
    """Exhaustive FP64 requests scored by Cholesky columns with different
    design sizes, lengthscales and nuggets share one batch (one launch with
    per-location parameters): each request's results equal the oracle's own
    run of it."""
    rng = np.random.default_rng(531)
    X = rng.random((50000, 4))
    y = W.f_mix4(X)
    base = W.Params(n0=6, ncand=1000, scoring=W.SCORING_CHOL)
    prms = [base.replace(n=n, d=(d,), g=g) for n, d, g in
            [(20, 0.1, 1e-6), (50, 0.05, 1e-4), (35, 0.2, 1e-6), (50, 0.1, 1e-6), (8, 0.1, 1e-2), (41, 0.3, 0.0)]]
    reqs = [(rng.random((int(m), 4)), prm) for m, prm in zip([7, 13, 1, 30, 5, 9], prms)]
    import torch

    d = lg.Design(torch.from_numpy(X), torch.from_numpy(y))
    srv = lg.lagp_server_create(d.handle, 4 << 30, 1)  # one slot: the requests wait and batch together
    try:
        tickets = [lg.lagp_server_submit(srv, XX, lg.make_params(prm))[1] for XX, prm in reqs]
        res = [lg.lagp_server_fetch(srv, t, XX.shape[0], prm.n) for t, (XX, prm) in zip(tickets, reqs)]
    finally:
        lg.lagp_server_destroy(srv)
        d.close()
    for k, ((XX, prm), r) in enumerate(zip(reqs, res)):
        _same(r, oracle.predict(X, y, XX, prm), f"request {k}")


@pytest.mark.parametrize("p,R,n", [(8, 1, 50), (8, 7, 50), (2, 16, 64), (3, 17, 40), (8, 10, 64)])
def test_ray_tile_and_wave_forms_bit_exact(lg, monkeypatch, p, R, n):
    """Up to 16 rays at n <= 64 run on one wave per location (every ray on a
    lane, each round one tile of the exact scoring); LAGP_RAY_FORCE_WAVES=1
    keeps the four-wave form.  Both equal the oracle bit for bit, Brent
    evaluation counts included (R = 17 takes the four-wave form either way)."""
    import torch

    w = _uniform(540 + p + R, 20000, p, 6, n0=6, n=n, ncand=600, search=W.SEARCH_RAY, numrays=R, d=(0.15 * p,),
                 g=1e-6)
    o = oracle.predict(w.X, w.y, w.XX, w.params)
    runs = []
    for force in ("0", "1"):
        monkeypatch.setenv("LAGP_RAY_FORCE_WAVES", force)
        d = lg.Design(torch.from_numpy(w.X), torch.from_numpy(w.y))
        try:
            out = d.predict(torch.from_numpy(w.XX), w.params, counts=True)
            torch.cuda.synchronize()
            g = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
        finally:
            d.close()
        _same(g, o, f"rays p={p} R={R} n={n} force_waves={force}")
        assert np.array_equal(g["diag"][:, :, 0], o["diag"][:, :, 1])
        assert np.array_equal(g["counts"][:, :, 0], o["diag"][:, :, 5].astype(np.int32))
        runs.append(g)
    for k in ("sel", "mean", "s2", "diag", "counts"):
        assert np.array_equal(runs[0][k], runs[1][k]), k
