"""Continuous-batching server through the C ABI (MI355X only): every
request's results are the same alone, in a mix and as a direct
lagp_predict call; admission respects the HBM budget."""
import threading

import numpy as np
import pytest

from paper_1409_0074_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1409_0074_amd as lg

    assert torch.cuda.is_available()
    rng = np.random.default_rng(201)
    X = rng.random((200_000, 4))
    y = W.f_mix4(X)
    d = lg.Design(torch.from_numpy(X), torch.from_numpy(y))
    yield lg, d, rng
    d.close()


def _requests(rng, count):
    out = []
    for k in range(count):
        m = int(np.floor(10 ** rng.uniform(0, 2.5)))
        n = [30, 50, 100][k % 3]
        search = W.SEARCH_RAY if k % 2 else W.SEARCH_EXHAUSTIVE
        chol = search == W.SEARCH_EXHAUSTIVE and n <= 50 and k % 4 == 0  # both scoring forms in the mix
        prm = W.Params(n0=6, n=n, ncand=1000 if n < 100 else 1200, search=search, numrays=4, d=(0.1,), g=1e-6,
                       scoring=W.SCORING_CHOL if chol else W.SCORING_PARTINV)
        out.append((rng.random((m, 4)), prm))
    return out


def _direct(lg, d, XX, prm):
    import torch

    o = d.predict(torch.from_numpy(XX), prm, diag=False)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items() if v is not None}


def _serve(lg, d, reqs, budget=8 << 30, slots=4):
    srv = lg.lagp_server_create(d.handle, budget, slots)
    try:
        tickets = []
        for XX, prm in reqs:
            rc, t = lg.lagp_server_submit(srv, XX, lg.make_params(prm))
            assert rc == lg.LAGP_OK
            tickets.append(t)
        res = [lg.lagp_server_fetch(srv, t, XX.shape[0], prm.n) for t, (XX, prm) in zip(tickets, reqs)]
        stats = lg.lagp_server_stats(srv)
    finally:
        lg.lagp_server_destroy(srv)
    return res, stats


def _same(a, b):
    assert np.array_equal(a["sel"], b["sel"])
    assert np.array_equal(a["mean"], b["mean"]) and np.array_equal(a["s2"], b["s2"])
    assert np.array_equal(a["status"], b["status"])


def test_mix_equals_alone_equals_direct(env):
    lg, d, rng = env
    reqs = _requests(rng, 18)
    mixed, stats = _serve(lg, d, reqs)
    assert stats["p99_ms"] >= stats["p50_ms"] > 0 and stats["pred_per_s"] > 0
    for k in (0, 3, 7, 11):
        alone, _ = _serve(lg, d, [reqs[k]])
        _same(mixed[k], alone[0])
    for k, (XX, prm) in enumerate(reqs):
        _same(mixed[k], _direct(lg, d, XX, prm))


def test_tiny_budget_serialises_but_completes(env):
    lg, d, rng = env
    reqs = _requests(rng, 6)
    # room for about one request at a time
    budget = 64 << 20
    res, _ = _serve(lg, d, reqs, budget=budget, slots=3)
    for (XX, prm), r in zip(reqs, res):
        _same(r, _direct(lg, d, XX, prm))


def test_concurrent_submitters(env):
    lg, d, rng = env
    reqs = _requests(rng, 12)
    srv = lg.lagp_server_create(d.handle, 4 << 30, 4)
    results = [None] * len(reqs)

    def client(ks):
        for k in ks:
            XX, prm = reqs[k]
            _, t = lg.lagp_server_submit(srv, XX, lg.make_params(prm))
            results[k] = lg.lagp_server_fetch(srv, t, XX.shape[0], prm.n)

    th = [threading.Thread(target=client, args=(list(range(i, len(reqs), 3)),)) for i in range(3)]
    [t.start() for t in th]
    [t.join() for t in th]
    lg.lagp_server_destroy(srv)
    for (XX, prm), r in zip(reqs, results):
        _same(r, _direct(lg, d, XX, prm))


def test_oversized_and_invalid_requests(env):
    lg, d, rng = env
    srv = lg.lagp_server_create(d.handle, 2 << 20, 1)
    try:
        with pytest.raises(lg.LagpError) as e:
            lg.lagp_server_submit(srv, rng.random((500, 4)), lg.make_params(W.Params(n=50, ncand=1000, d=(0.1,))))
        assert e.value.code == lg.LAGP_ENOMEM
        with pytest.raises(lg.LagpError) as e:
            lg.lagp_server_submit(srv, rng.random((5, 4)), lg.make_params(W.Params(n=50, ncand=10, d=(0.1,))))
        assert e.value.code == lg.LAGP_EINVAL
    finally:
        lg.lagp_server_destroy(srv)
