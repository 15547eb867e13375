"""Pins of the CPU oracle against things other than itself: the mathematics
of Secs. 2-4 of the paper, brute force on tiny inputs, exact arithmetic,
library routines and hand-worked values.  CPU only."""
import math
import os
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

from paper_1409_0074_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _gauss(A, B, d):
    """Plain Gaussian correlation matrix exp(-sum_k (a_k-b_k)^2/d_k) in numpy."""
    d = np.broadcast_to(np.atleast_1d(d), (A.shape[1],))
    D = ((A[:, None, :] - B[None, :, :]) ** 2 / d).sum(-1)
    return np.exp(-D)


def _fma_exact(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


# ----------------------------------------------------------------- pieces --

def test_exp_is_faithful(orc):
    """The oracle's exp is within one ulp of exp computed to 150 bits."""
    mp.mp.prec = 150
    rng = np.random.default_rng(5)
    xs = np.concatenate([-rng.random(1500) * 708.0, -rng.random(1500) * 4.0, [0.0, -1e-300, -707.999, -0.5]])
    for x in xs:
        ref = mp.exp(mp.mpf(float(x)))
        err = abs(mp.mpf(orc.exp(x)) - ref) / np.spacing(float(ref))
        assert err <= 1.0, (x, float(err))
    assert orc.exp(-709.0) == 0.0  # below the flush threshold


def test_sqdist_is_the_defined_fma_chain(orc):
    """Squared distance = fma(t_k, t_k, s) in dimension order, each step
    rounded once; checked with exact rational arithmetic."""
    rng = np.random.default_rng(6)
    for _ in range(300):
        p = int(rng.integers(1, 9))
        a, b = rng.random(p), rng.random(p)
        s = 0.0
        for k in range(p):
            t = float(a[k] - b[k])
            s = _fma_exact(t, t, s)
        assert orc.sqdist(a, b) == s


def test_kernel_closed_form(orc):
    rng = np.random.default_rng(7)
    for _ in range(200):
        p = int(rng.integers(1, 9))
        a, b = rng.random(p), rng.random(p)
        d = 0.05 + rng.random()
        ref = math.exp(-sum((a - b) ** 2) / d)
        assert orc.kern(a, b, [d]) == pytest.approx(ref, rel=4e-15, abs=1e-300)
        dk = 0.05 + rng.random(p)
        ref = math.exp(-sum((a - b) ** 2 / dk))
        assert orc.kern(a, b, dk) == pytest.approx(ref, rel=4e-15, abs=1e-300)
    assert orc.kern([0.3, 0.4], [0.3, 0.4], [0.1]) == 1.0


def test_spd_inverse_vs_numpy(orc):
    rng = np.random.default_rng(8)
    for n in (1, 2, 6, 12):
        X = rng.random((n, 2))
        A = _gauss(X, X, 0.1) + 1e-3 * np.eye(n)
        Ai = orc.spd_inverse(A)
        ref = np.linalg.inv(A)
        assert np.abs(Ai - ref).max() <= 1e-10 * np.abs(ref).max()
    with pytest.raises(np.linalg.LinAlgError):
        orc.spd_inverse(np.array([[1.0, 2.0], [2.0, 1.0]]))


# ------------------------------------------------------------------- kNN --

def _knn_brute(X, x, ncand):
    """Exactly-rounded defined distances, ordered by (d2, row) with sorted()."""
    d2 = []
    for i in range(X.shape[0]):
        s = 0.0
        for k in range(X.shape[1]):
            t = float(X[i, k] - x[k])
            s = _fma_exact(t, t, s)
        d2.append((s, i))
    d2.sort()
    return [i for _, i in d2[:ncand]], [s for s, _ in d2[:ncand]]


def test_knn_vs_sorted_bruteforce(orc):
    rng = np.random.default_rng(9)
    X = rng.random((257, 3))
    XX = rng.random((4, 3))
    idx, d2 = orc.knn(X, XX, 40, nthreads=2)
    for m in range(4):
        bi, bd = _knn_brute(X, XX[m], 40)
        assert list(idx[m]) == bi
        assert list(d2[m]) == bd


def test_knn_ties_go_to_lower_row(orc):
    """On a grid, many rows share a distance; ties are broken by row index."""
    X = W.grid2(11)
    x = np.array([0.5, 0.5])  # a grid point: rings of equal distance around it
    idx, d2 = orc.knn(X, x[None], 21, nthreads=1)
    bi, bd = _knn_brute(X, x, 21)
    assert list(idx[0]) == bi
    assert list(d2[0]) == bd
    assert len(set(d2[0])) < 21  # the case really has ties
    assert np.all(np.diff(d2[0]) >= 0)


# --------------------------------------------------- greedy design (exh) --

def _bracket(Xd, J, x, g, d):
    """b = (1+g) - k_x^T (K_J + g I)^{-1} k_x from a fresh solve."""
    XJ = Xd[J]
    K = _gauss(XJ, XJ, d) + g * np.eye(len(J))
    kx = _gauss(XJ, x[None], d)[:, 0]
    return (1.0 + g) - kx @ np.linalg.solve(K, kx)


@pytest.mark.parametrize("g,d,rtol", [(1e-3, 0.1, 1e-8), (1e-3, 0.5, 1e-8), (1e-4, 0.2, 1e-5)])
def test_alc_equals_fresh_variance_reduction(orc, g, d, rtol):
    """Every candidate's score at every step equals the reduction of the
    kriging bracket at x when that candidate joins the design, with both
    brackets from freshly solved systems (Sec. 3.1, Eq. alc integrand)."""
    rng = np.random.default_rng(10)
    X = rng.random((140, 2))
    y = W.f_bump2(X)
    x = np.array([0.41, 0.57])
    prm = W.Params(n0=4, n=16, ncand=140, d=(d,), g=g)
    tr = orc.trace(X, y, x, prm)
    cand = tr["cand"]
    sel = list(tr["sel"])
    for step in range(prm.n - prm.n0):
        j = prm.n0 + step
        J = sel[:j]
        b = _bracket(X, J, x, g, d)
        alc = tr["alc"][step]
        checked = 0
        for q in range(0, 140, 7):
            r = int(cand[q])
            if r in J:
                assert np.isnan(alc[q])
                continue
            red = b - _bracket(X, J + [r], x, g, d)
            # both sides carry ~eps*cond(K) error: the oracle through the explicit
            # inverse's quadratic form (8.7e-9 relative at g = 1e-4 on an early
            # step, checked against 50-digit arithmetic), the brute force through
            # b - b'; a dropped term or wrong sign is an O(1) error
            assert abs(alc[q] - red) <= rtol * abs(red) + 1e-10 * b, (step, q, alc[q], red)
            checked += 1
        assert checked > 0


def test_alc_matches_papers_expanded_integrand(orc):
    """The integrand of Eq. alc written out term by term, with
    g_j = -K^{-1} k_j(x_c)/v_j (the sign the partitioned inverse needs)."""
    rng = np.random.default_rng(11)
    X = rng.random((120, 2))
    y = W.f_bump2(X)
    x = np.array([0.3, 0.6])
    g, d = 1e-3, 0.2
    prm = W.Params(n0=5, n=12, ncand=120, d=(d,), g=g)
    tr = orc.trace(X, y, x, prm)
    sel, cand = list(tr["sel"]), tr["cand"]
    step = 4
    J = sel[: prm.n0 + step]
    XJ = X[J]
    K = _gauss(XJ, XJ, d) + g * np.eye(len(J))
    Ki = np.linalg.inv(K)
    kx = _gauss(XJ, x[None], d)[:, 0]
    for q in range(120):
        r = int(cand[q])
        if r in J:
            continue
        kc = _gauss(XJ, X[r][None], d)[:, 0]
        v = (1.0 + g) - kc @ Ki @ kc
        gj = -(Ki @ kc) / v
        G = np.outer(gj, gj)
        Kcx = _gauss(X[r][None], x[None], d)[0, 0]
        terms = (kx @ G @ kx * v, 2.0 * (kx @ gj) * Kcx, Kcx ** 2 / v)
        integrand = sum(terms)
        # the three terms cancel; their rounding error scales with the largest
        assert abs(tr["alc"][step][q] - integrand) <= 1e-10 * max(abs(t) for t in terms) + 1e-15


def test_partitioned_inverse_vs_direct_inverse(orc):
    """The inverse grown by partitioned-inverse updates (Sec. 3.1) equals the
    direct inverse of K_J + g I.  The update recurrence loses accuracy as the
    nugget shrinks (Schur complements v ~ g cancel): against a 50-digit
    inverse it is 2e-10 off at g = 1e-3 (cond 2e4), 1e-4 at g = 1e-6 (cond
    1.8e7) and useless at g = 1e-10, while a direct inverse stays near
    eps*cond.  Strict at g = 1e-3; a regression guard at g = 1e-6."""
    rng = np.random.default_rng(12)
    X = rng.random((400, 2))
    y = W.f_bump2(X)
    for g, bound in ((1e-3, None), (1e-6, 1e-3), (1e-10, None)):
        prm = W.Params(n0=6, n=30, ncand=200, d=(0.1,), g=g)
        tr = orc.trace(X, y, np.array([0.5, 0.45]), prm)
        XJ = X[tr["sel"]]
        K = _gauss(XJ, XJ, 0.1) + g * np.eye(30)
        ref = np.linalg.inv(K)
        err = np.abs(tr["Ki"] - ref).max() / np.abs(ref).max()
        assert np.array_equal(tr["Ki"], tr["Ki"].T)  # the update keeps exact symmetry
        if g == 1e-3:
            assert err <= 100 * np.finfo(float).eps * np.linalg.cond(K), err
        elif bound is not None:
            assert err <= bound, (g, err)


def test_exhaustive_choice_is_bruteforce_argmax(orc):
    """The oracle's pick is the argmax of the brute-force reductions."""
    rng = np.random.default_rng(13)
    X = rng.random((150, 2))
    y = W.f_bump2(X)
    x = np.array([0.62, 0.33])
    g, d = 1e-3, 0.15
    prm = W.Params(n0=6, n=14, ncand=150, d=(d,), g=g)
    tr = orc.trace(X, y, x, prm)
    sel = list(tr["sel"])
    for step in range(prm.n - prm.n0):
        J = sel[: prm.n0 + step]
        b = _bracket(X, J, x, g, d)
        reds = {r: b - _bracket(X, J + [r], x, g, d) for r in range(150) if r not in J}
        order = sorted(reds.items(), key=lambda kv: -kv[1])
        if (order[0][1] - order[1][1]) > 1e-8 * order[0][1]:
            assert sel[prm.n0 + step] == order[0][0]


@pytest.mark.parametrize("g", [1e-6, 1e-3])
def test_invariants_alc_nonneg_and_bracket_decreasing(orc, g):
    """ALC >= 0 for every scored candidate; the kriging bracket b_j at x never
    grows, and drops by exactly the chosen candidate's score."""
    w = W.tiny_2d(M=12)
    prm = w.params.replace(g=g)
    out = orc.predict(w.X, w.y, w.XX, prm, nthreads=4)
    dg = out["diag"]
    assert np.all(dg[:, :, 1] >= 0.0) and np.all(dg[:, :, 3] >= 0.0)
    b = dg[:, :, 6]
    # b_j is a quadratic form in K^{-1}, whose norm is at most 1/g: its
    # absolute rounding error is of order eps * n / g
    tol = 10.0 * np.finfo(float).eps * prm.n / g
    assert np.all(np.diff(b, axis=1) <= tol)
    assert np.all(b >= g - tol)
    drop = b[:, :-1] - b[:, 1:]
    assert np.allclose(drop, dg[:, :-1, 3], rtol=1e-6, atol=tol)
    tr = orc.trace(w.X, w.y, w.XX[0], prm)
    a = tr["alc"]
    assert np.nanmin(a) >= 0.0


def test_full_design_reproduces_full_gp(orc):
    """n = N' = N: the local design holds every point, so the prediction is
    the full GP's (Eqs. predgp, preds2 with N points), in any order."""
    rng = np.random.default_rng(14)
    N = 48
    X = rng.random((N, 2))
    y = W.f_bump2(X)
    XX = rng.random((5, 2))
    g, d = 1e-3, 0.1
    prm = W.Params(n0=3, n=N, ncand=N, d=(d,), g=g)
    out = orc.predict(X, y, XX, prm, nthreads=2)
    K = _gauss(X, X, d) + g * np.eye(N)
    psi = y @ np.linalg.solve(K, y)
    for m in range(5):
        k = _gauss(X, XX[m][None], d)[:, 0]
        mu = k @ np.linalg.solve(K, y)
        s2 = psi * ((1.0 + g) - k @ np.linalg.solve(K, k)) / N
        assert out["mean"][m] == pytest.approx(mu, rel=1e-9, abs=1e-12)
        assert out["s2"][m] == pytest.approx(s2, rel=1e-7)
        assert sorted(out["sel"][m]) == list(range(N))
        assert out["df"][m] == N


def test_nn_mode_is_nearest_neighbour_kriging(orc):
    rng = np.random.default_rng(15)
    X = rng.random((500, 2))
    y = W.f_bump2(X)
    XX = rng.random((4, 2))
    g, d, n = 1e-4, 0.1, 20
    prm = W.Params(n0=n, n=n, ncand=n, search=W.SEARCH_NN, d=(d,), g=g)
    out = orc.predict(X, y, XX, prm, nthreads=2)
    for m in range(4):
        J = np.argsort(((X - XX[m]) ** 2).sum(1), kind="stable")[:n]
        K = _gauss(X[J], X[J], d) + g * np.eye(n)
        k = _gauss(X[J], XX[m][None], d)[:, 0]
        assert out["mean"][m] == pytest.approx(k @ np.linalg.solve(K, y[J]), rel=1e-9, abs=1e-12)
        assert sorted(out["sel"][m]) == sorted(J)


def test_design_ignores_responses_and_scales(orc):
    """The local design depends on X only (Sec. 2.2); under y -> a y the mean
    scales by a and the scale by a^2."""
    w = W.tiny_2d(M=6)
    o1 = orc.predict(w.X, w.y, w.XX, w.params, nthreads=2)
    o2 = orc.predict(w.X, -3.0 * w.y + 0.0, w.XX, w.params, nthreads=2)
    o3 = orc.predict(w.X, np.cos(w.y * 7.0), w.XX, w.params, nthreads=2)
    assert np.array_equal(o1["sel"], o2["sel"]) and np.array_equal(o1["sel"], o3["sel"])
    assert np.allclose(o2["mean"], -3.0 * o1["mean"], rtol=1e-12, atol=1e-15)
    assert np.allclose(o2["s2"], 9.0 * o1["s2"], rtol=1e-12)


def test_row_permutation_selects_same_points(orc):
    w = W.tiny_2d(M=5)
    perm = np.random.default_rng(16).permutation(w.X.shape[0])
    o1 = orc.predict(w.X, w.y, w.XX, w.params, nthreads=2)
    o2 = orc.predict(w.X[perm], w.y[perm], w.XX, w.params, nthreads=2)
    for m in range(5):
        a = [tuple(v) for v in w.X[o1["sel"][m]]]
        b = [tuple(v) for v in w.X[perm][o2["sel"][m]]]
        assert a == b
    assert np.allclose(o1["mean"], o2["mean"], rtol=1e-13, atol=1e-15)


def test_replay_of_own_sequence_is_identity(orc):
    w = W.tiny_2d(M=6)
    o1 = orc.predict(w.X, w.y, w.XX, w.params, nthreads=2)
    o2 = orc.predict(w.X, w.y, w.XX, w.params, forced=o1["sel"], nthreads=2)
    assert np.array_equal(o1["sel"], o2["sel"])
    assert np.array_equal(o1["mean"], o2["mean"]) and np.array_equal(o1["s2"], o2["s2"])
    assert np.array_equal(o2["diag"][:, :, 0], o1["sel"][:, w.params.n0:].astype(float))


def test_oracle_fp64_error_vs_high_precision(orc):
    """Tiny case recomputed in 60-digit arithmetic on the oracle's own design."""
    mp.mp.dps = 60
    rng = np.random.default_rng(17)
    X = rng.random((80, 2))
    y = W.f_bump2(X)
    x = np.array([0.47, 0.52])
    g, d = 1e-3, 0.1
    prm = W.Params(n0=4, n=12, ncand=80, d=(d,), g=g)
    out = orc.predict(X, y, x[None], prm, nthreads=1)
    J = out["sel"][0]
    XJ = [[mp.mpf(float(v)) for v in X[i]] for i in J]
    xm = [mp.mpf(float(v)) for v in x]

    def kk(a, b):
        return mp.exp(-sum((ai - bi) ** 2 for ai, bi in zip(a, b)) / mp.mpf(d))

    n = len(J)
    K = mp.matrix(n, n)
    for i in range(n):
        for k in range(n):
            K[i, k] = kk(XJ[i], XJ[k]) + (mp.mpf(g) if i == k else 0)
    kx = mp.matrix([kk(XJ[i], xm) for i in range(n)])
    yJ = mp.matrix([mp.mpf(float(y[i])) for i in J])
    Ki = K ** -1
    mu = (kx.T * Ki * yJ)[0]
    psi = (yJ.T * Ki * yJ)[0]
    s2 = psi * (1 + mp.mpf(g) - (kx.T * Ki * kx)[0]) / n
    assert abs(out["mean"][0] - float(mu)) <= 1e-11 * abs(float(mu)) + 1e-14
    assert abs(out["s2"][0] - float(s2)) <= 1e-9 * float(s2)


# ------------------------------------------------------------ ray search --

def test_ray_k0_golden(orc):
    rows = np.loadtxt(os.path.join(GOLDEN, "ray_k0.txt"), dtype=int)
    for t, k in rows:
        assert orc.ray_k0(t) == k, t


def test_ray_segment_golden(orc):
    rows = np.loadtxt(os.path.join(GOLDEN, "ray_segments.txt"))
    lo, hi = np.zeros(2), np.ones(2)
    for a1, a2, x1, x2, tau, d1, d2 in rows:
        t, d = orc.ray_segment([a1, a2], [x1, x2], lo, hi)
        assert t == pytest.approx(tau, abs=1e-12)
        assert d == pytest.approx([d1, d2], abs=1e-12)


@pytest.mark.parametrize("f,xstar", [
    (lambda s: (s - 0.3) ** 2, 0.3),
    (lambda s: (s - 0.71) ** 4 + 0.1, 0.71),
    (lambda s: -math.sin(math.pi * s) * math.exp(-s), math.atan(math.pi) / math.pi),
    (lambda s: abs(s - 0.123), 0.123),
    (lambda s: s * s * s - s, 1.0 / math.sqrt(3.0)),
])
def test_brent_finds_analytic_minimisers(orc, f, xstar):
    tol = 2.0 ** -13
    x, fx, ne, _ = orc.brent_min(f, 0.0, 1.0, tol, 100)
    assert abs(x - xstar) <= 3 * tol
    assert fx == f(x)
    assert ne < 60


def test_brent_matches_scipy_bounded(orc):
    """scipy's bounded minimiser is also Brent's method: same minimiser."""
    from scipy.optimize import minimize_scalar

    rng = np.random.default_rng(18)
    for _ in range(20):
        c = rng.random(3)
        f = lambda s: math.cos(6.0 * s * c[0] + c[1]) + (s - c[2]) ** 2  # noqa: E731
        x, _, _, _ = orc.brent_min(f, 0.0, 1.0, 1e-10, 200)
        r = minimize_scalar(f, bounds=(0.0, 1.0), method="bounded", options={"xatol": 1e-10})
        assert abs(f(x) - r.fun) <= 1e-12 or abs(x - r.x) <= 1e-6


@pytest.mark.parametrize("c", [0.3, 0.05, 0.77, 0.5])
def test_brent_parabolic_step_on_quadratic(orc, c):
    """On a parabola the interpolation step lands on the minimiser at once:
    Brent's method then needs as few evaluations as scipy's bounded Brent
    (6 here); golden-section search alone would need about 20."""
    from scipy.optimize import minimize_scalar

    f = lambda s: (s - c) ** 2 + 1.0  # noqa: E731
    x, _, ne, _ = orc.brent_min(f, 0.0, 1.0, 2.0 ** -13, 100)
    r = minimize_scalar(f, bounds=(0.0, 1.0), method="bounded", options={"xatol": 2.0 ** -13})
    assert abs(x - c) <= 1e-12
    assert ne <= r.nfev


def test_brent_boundary_minimum(orc):
    x, _, _, _ = orc.brent_min(lambda s: s, 0.0, 1.0, 2.0 ** -13, 100)
    assert x <= 3 * 2.0 ** -13


def _ray_starts(cand, inJ_rows, k0, R):
    rem = [q for q in range(len(cand)) if int(cand[q]) not in inJ_rows]
    return rem[k0:k0 + R]


@pytest.mark.parametrize("snap", [W.SNAP_CANDIDATES, W.SNAP_DESIGN])
def test_ray_step_snap_bruteforce(orc, snap):
    """Recompute each ray step's start ranks, segments and snap in numpy from
    the oracle's own reported s* and check the chosen candidate (Sec. 4);
    with the whole-design scope (Sec. 5) the snap must reach the nearest of
    all design rows outside the design and the starts."""
    w = W.tiny_2d(M=8)
    prm = w.params.replace(search=W.SEARCH_RAY, numrays=3, n=30, snap=snap)
    lo, hi = w.X.min(0), w.X.max(0)
    for m in range(8):
        x = w.XX[m]
        tr = orc.trace(w.X, w.y, x, prm)
        cand, sel, dg = tr["cand"], list(tr["sel"]), tr["diag"]
        for step in range(prm.n - prm.n0):
            j = prm.n0 + step
            J = set(int(v) for v in sel[:j])
            starts = _ray_starts(cand, J, orc.ray_k0(step + 1), 3)
            s_win = dg[step, 7]
            chosen = sel[j]
            # the s = 0 post-check makes every ray worth at least its start;
            # the starts' scores come from the exhaustive candidate trace
            start_alc = max(tr["alc"][step][q] for q in starts)
            assert dg[step, 1] >= start_alc * (1.0 - 1e-9), (m, step)
            if s_win == 0.0:
                assert chosen in [int(cand[q]) for q in starts]
                q = [int(cand[r]) for r in starts].index(chosen)
                assert tr["alc"][step][starts[q]] == pytest.approx(dg[step, 1], rel=1e-9)
                continue
            # a snapped point is never one of this step's ray starts
            assert chosen not in [int(cand[q]) for q in starts], (m, step)
            # which ray: the one whose segment contains the snapped-from point
            best = None
            for q in starts:
                a = w.X[cand[q]]
                _, dvec = orc.ray_segment(a, x, lo, hi)
                z = a + s_win * dvec
                allowed = [int(cand[r]) for r in range(len(cand)) if int(cand[r]) not in J and r not in starts]
                dd = ((w.X[allowed] - z) ** 2).sum(1)
                nearest = allowed[int(np.argmin(dd))]
                if nearest == chosen:
                    best = q
            assert best is not None, (m, step)
        if snap == W.SNAP_DESIGN:
            assert len(cand) == w.X.shape[0]


def test_ray_mode_predicts_well(orc):
    """Rays trade a little accuracy for time (Sec. 5); on the 2-d bump both
    modes land close to the truth."""
    w = W.tiny_2d(M=40)
    ex = orc.predict(w.X, w.y, w.XX, w.params, nthreads=4)
    ry = orc.predict(w.X, w.y, w.XX, w.params.replace(search=W.SEARCH_RAY, numrays=2), nthreads=4)
    rm_ex = np.sqrt(np.mean((ex["mean"] - w.truth) ** 2))
    rm_ry = np.sqrt(np.mean((ry["mean"] - w.truth) ** 2))
    assert rm_ex < 1e-3 and rm_ry < 1e-3
    assert np.all(ry["status"] == 0)


def test_local_designs_mix_neighbours_and_satellites(orc):
    """Fig. 1: greedy local designs at x = (-1.725, 1.725) on the 201 x 201
    grid over [-2,2]^2 mix nearest neighbours with farther satellite points.
    The paper shows roughly a 2:1 split but not its parameters; checked
    loosely."""
    g1 = np.linspace(-2.0, 2.0, 201)
    a, b = np.meshgrid(g1, g1, indexing="ij")
    X = np.stack([a.ravel(), b.ravel()], 1)
    y = np.zeros(X.shape[0])
    x = np.array([-1.725, 1.725])
    prm = W.Params(n0=6, n=50, ncand=1000, d=(0.5,), g=1e-6)
    out = orc.predict(X, y, x[None], prm, nthreads=4)
    nn50 = set(np.argsort(((X - x) ** 2).sum(1), kind="stable")[:50].tolist())
    frac = np.mean([int(r) in nn50 for r in out["sel"][0]])
    assert 0.3 <= frac <= 0.95, frac


def test_golden_fixture_is_reproduced(orc):
    """Bit-for-bit regression guard written by tests/golden/make_golden.py
    (oracle only): any change to the oracle's arithmetic shows up here."""
    import json

    with open(os.path.join(GOLDEN, "oracle_uniform2d.json")) as f:
        gold = json.load(f)
    w = W.tiny_2d(M=8)
    for tag, prm in (("exhaustive", w.params), ("ray2", w.params.replace(search=W.SEARCH_RAY, numrays=2))):
        r = orc.predict(w.X, w.y, w.XX, prm, nthreads=3)
        assert r["sel"].tolist() == gold[tag]["sel"]
        assert [float(v).hex() for v in r["mean"]] == gold[tag]["mean"]
        assert [float(v).hex() for v in r["s2"]] == gold[tag]["s2"]


def test_singular_start_reports_nan(orc):
    """Duplicate design rows with no nugget make the starting covariance
    singular: the location reports NaN and the NOTPD status bit."""
    X = np.repeat(np.random.default_rng(19).random((50, 2)), 2, axis=0)
    y = W.f_bump2(X)
    prm = W.Params(n0=4, n=8, ncand=20, d=(0.1,), g=0.0)
    out = orc.predict(X, y, X[:3] + 0.0, prm, nthreads=1)
    assert np.all(np.isnan(out["mean"])) and np.all(out["status"] & orc.STATUS_NOTPD)
    assert np.all(out["sel"][:, 4:] == -1)


# ---------------------------------------------- Cholesky form of the search --

def _mp_alc_all(X, x, J, cands, d, g):
    """Integrand of Eq. alc at x for each candidate row, with 40-digit
    arithmetic on the design J (Cholesky solves in mpmath)."""
    mp.mp.dps = 40
    P = {int(r): [mp.mpf(float(v)) for v in X[r]] for r in list(J) + list(cands)}
    xm = [mp.mpf(float(v)) for v in x]

    def kk(a, b):
        return mp.exp(-sum((ai - bi) ** 2 for ai, bi in zip(a, b)) / mp.mpf(d))

    n = len(J)
    K = mp.matrix(n, n)
    for i in range(n):
        for k in range(n):
            K[i, k] = kk(P[int(J[i])], P[int(J[k])]) + (mp.mpf(g) if i == k else 0)
    L = mp.cholesky(K)

    def fsolve(b):
        z = []
        for i in range(n):
            s = b[i]
            for k in range(i):
                s -= L[i, k] * z[k]
            z.append(s / L[i, i])
        return z

    w = fsolve([kk(P[int(J[i])], xm) for i in range(n)])
    out = []
    for r in cands:
        u = fsolve([kk(P[int(J[i])], P[int(r)]) for i in range(n)])
        v = 1 + mp.mpf(g) - sum(ui * ui for ui in u)
        c = kk(P[int(r)], xm) - sum(ui * wi for ui, wi in zip(u, w))
        out.append(float(c * c / v))
    return np.array(out)


def test_chol_form_equals_partitioned_form_when_well_conditioned(orc):
    """With a large nugget both forms are accurate to ~1e-12, so they must
    choose the same designs and agree in every criterion value and in the
    prediction (O7 against O4-O6)."""
    w = W.tiny_2d(M=8)
    prm = w.params.replace(g=1e-2, n=30)
    a = orc.predict(w.X, w.y, w.XX, prm, nthreads=2)
    b = orc.predict(w.X, w.y, w.XX, prm.replace(scoring=W.SCORING_CHOL), nthreads=2)
    assert np.array_equal(a["sel"], b["sel"])
    assert np.allclose(b["mean"], a["mean"], rtol=1e-10, atol=1e-14)
    assert np.allclose(b["s2"], a["s2"], rtol=1e-10, atol=0)
    assert np.allclose(b["diag"][:, :, 1], a["diag"][:, :, 1], rtol=1e-9, atol=0)
    assert np.all(b["status"] == 0)
    ta = orc.trace(w.X, w.y, w.XX[0], prm)
    tb = orc.trace(w.X, w.y, w.XX[0], prm.replace(scoring=W.SCORING_CHOL))
    fin = np.isfinite(ta["alc"])
    assert np.array_equal(fin, np.isfinite(tb["alc"]))
    for step in range(ta["alc"].shape[0]):
        f = fin[step]
        top = np.max(ta["alc"][step][f])
        assert np.allclose(tb["alc"][step][f], ta["alc"][step][f], rtol=1e-8, atol=1e-10 * top), step


def test_chol_form_vs_high_precision_at_small_nugget(orc):
    """g = 1e-6: v_c sits near g at late steps, so FP64 criterion values
    lose digits in proportion to 1/v_c.  The Cholesky form's values stay
    within 1e-6 of 40-digit arithmetic on every step, its choice is the
    40-digit argmax wherever the top two differ by more than 1e-6, and its
    prediction is within 1e-9 (mean) / 1e-7 (scale) of 40-digit values."""
    rng = np.random.default_rng(21)
    X = rng.random((300, 2))
    y = W.f_bump2(X)
    x = np.array([0.43, 0.55])
    d, g = 0.1, 1e-6
    prm = W.Params(n0=4, n=20, ncand=80, d=(d,), g=g, scoring=W.SCORING_CHOL)
    tr = orc.trace(X, y, x, prm)
    cand, sel = tr["cand"], list(tr["sel"])
    worst = 0.0
    for step in range(prm.n - prm.n0):
        j = prm.n0 + step
        free = [q for q in range(prm.ncand) if int(cand[q]) not in sel[:j]]
        hp = _mp_alc_all(X, x, sel[:j], [cand[q] for q in free], d, g)
        got = tr["alc"][step][free]
        worst = max(worst, float(np.max(np.abs(got - hp) / hp)))
        o = np.argsort(-hp)
        if (hp[o[0]] - hp[o[1]]) / hp[o[0]] > 1e-6:
            assert int(cand[free[o[0]]]) == sel[j], step
    assert worst <= 1e-6, worst
    mp.mp.dps = 40
    J = sel
    P = [[mp.mpf(float(v)) for v in X[r]] for r in J]
    xm = [mp.mpf(float(v)) for v in x]
    kk = lambda a, b: mp.exp(-sum((ai - bi) ** 2 for ai, bi in zip(a, b)) / mp.mpf(d))
    n = len(J)
    K = mp.matrix(n, n)
    for i in range(n):
        for k in range(n):
            K[i, k] = kk(P[i], P[k]) + (mp.mpf(g) if i == k else 0)
    kx = mp.matrix([kk(P[i], xm) for i in range(n)])
    yJ = mp.matrix([mp.mpf(float(y[r])) for r in J])
    a1, a2 = mp.lu_solve(K, kx), mp.lu_solve(K, yJ)
    mu = float(sum(a1[i] * yJ[i] for i in range(n)))
    s2 = float(sum(yJ[i] * a2[i] for i in range(n)) * (1 + mp.mpf(g) - sum(kx[i] * a1[i] for i in range(n))) / n)
    assert abs(tr["mean"] - mu) <= 1e-9 * abs(mu)
    assert abs(tr["s2"] - s2) <= 1e-7 * s2


def test_chol_form_full_design_reproduces_full_gp(orc):
    """n = N' = N: the Cholesky form's prediction is the full GP's."""
    rng = np.random.default_rng(22)
    N = 40
    X = rng.random((N, 2))
    y = W.f_bump2(X)
    XX = rng.random((4, 2))
    g, d = 1e-3, 0.1
    prm = W.Params(n0=2, n=N, ncand=N, d=(d,), g=g, scoring=W.SCORING_CHOL)
    out = orc.predict(X, y, XX, prm, nthreads=2)
    K = _gauss(X, X, d) + g * np.eye(N)
    psi = y @ np.linalg.solve(K, y)
    for m in range(4):
        k = _gauss(X, XX[m][None], d)[:, 0]
        assert out["mean"][m] == pytest.approx(k @ np.linalg.solve(K, y), rel=1e-9, abs=1e-12)
        assert out["s2"][m] == pytest.approx(psi * ((1.0 + g) - k @ np.linalg.solve(K, k)) / N, rel=1e-7)
        assert sorted(out["sel"][m]) == list(range(N))


def test_chol_form_start_only_is_nearest_neighbour_kriging(orc):
    """n0 = n: no greedy step; the factor of the n nearest gives their kriging
    prediction (Sec. 2.2)."""
    rng = np.random.default_rng(23)
    X = rng.random((500, 3))
    y = W.f_sines8(np.pad(X, ((0, 0), (0, 0))))
    XX = rng.random((4, 3))
    g, d, n = 1e-4, 0.3, 18
    prm = W.Params(n0=n, n=n, ncand=40, d=(d,), g=g, scoring=W.SCORING_CHOL)
    out = orc.predict(X, y, XX, prm, nthreads=2)
    for m in range(4):
        J = np.argsort(((X - XX[m]) ** 2).sum(1), kind="stable")[:n]
        K = _gauss(X[J], X[J], d) + g * np.eye(n)
        k = _gauss(X[J], XX[m][None], d)[:, 0]
        assert out["mean"][m] == pytest.approx(k @ np.linalg.solve(K, y[J]), rel=1e-9, abs=1e-12)
        assert list(out["sel"][m]) == list(J)


def test_chol_form_choice_is_argmax_of_its_scores(orc):
    """Every step takes the largest criterion among free candidates, lowest
    rank on ties, and records it."""
    w = W.tiny_2d(M=1)
    prm = w.params.replace(n=30, scoring=W.SCORING_CHOL)
    tr = orc.trace(w.X, w.y, w.XX[0], prm)
    for step in range(prm.n - prm.n0):
        a = np.where(np.isnan(tr["alc"][step]), -np.inf, tr["alc"][step])
        q = int(np.argmax(a))
        assert tr["sel"][prm.n0 + step] == tr["cand"][q]
        assert tr["diag"][step][1] == a[q]


def test_chol_form_singular_start(orc):
    X = np.repeat(np.random.default_rng(107).random((300, 2)), 2, axis=0)
    prm = W.Params(n0=4, n=10, ncand=40, d=(0.1,), g=0.0, scoring=W.SCORING_CHOL)
    out = orc.predict(X, W.f_bump2(X), X[:3].copy(), prm, nthreads=1)
    assert np.all(np.isnan(out["mean"])) and np.all(out["status"] & orc.STATUS_NOTPD)


# ------------------------------------------------- local MLE, two stages --

def _np_loglik(XJ, yJ, g, theta):
    """-1/2 log|K| - n/2 log(y^T K^{-1} y) written with numpy's determinant
    and solver (an implementation independent of the oracle's)."""
    n = len(yJ)
    K = _gauss(XJ, XJ, theta) + g * np.eye(n)
    sign, logdet = np.linalg.slogdet(K)
    assert sign > 0
    return -0.5 * logdet - 0.5 * n * np.log(yJ @ np.linalg.solve(K, yJ))


def _mle_case(seed, n=24, p=2):
    rng = np.random.default_rng(seed)
    XJ = rng.random((n, p)) * 0.4
    yJ = W.f_bump2(XJ) if p == 2 else W.f_sines8(np.pad(XJ, ((0, 0), (0, 8 - p))))
    return XJ, yJ


@pytest.mark.parametrize("seed", [41, 42, 43])
def test_mle_loglik_matches_numpy(orc, seed):
    XJ, yJ = _mle_case(seed)
    for theta in (0.01, 0.05, 0.3):
        l, _, _ = orc.mle_eval(XJ, yJ, 1e-4, theta)
        assert l == pytest.approx(_np_loglik(XJ, yJ, 1e-4, theta), rel=1e-9, abs=1e-9)


@pytest.mark.parametrize("seed", [41, 44])
def test_mle_derivatives_match_finite_differences(orc, seed):
    """l' and l'' (Eq. gpk differentiated) against central differences of
    numpy's log-likelihood and of the oracle's own l'."""
    XJ, yJ = _mle_case(seed)
    g = 1e-4
    for theta in (0.02, 0.08, 0.4):
        h = 1e-5 * theta
        l, d1, d2 = orc.mle_eval(XJ, yJ, g, theta)
        fd1 = (_np_loglik(XJ, yJ, g, theta + h) - _np_loglik(XJ, yJ, g, theta - h)) / (2 * h)
        assert d1 == pytest.approx(fd1, rel=1e-5, abs=1e-6 * abs(l) / theta)
        fd2 = (orc.mle_eval(XJ, yJ, g, theta + h)[1] - orc.mle_eval(XJ, yJ, g, theta - h)[1]) / (2 * h)
        assert d2 == pytest.approx(fd2, rel=1e-5, abs=1e-6 * abs(d1) / theta + 1e-3)


@pytest.mark.parametrize("seed", [41, 45, 46, 47])
def test_mle_fit_is_the_bruteforce_maximiser(orc, seed):
    """The safeguarded Newton estimate equals the maximiser of numpy's
    log-likelihood found by a log-spaced scan refined with scipy's bounded
    scalar search, to 1e-6 relative."""
    from scipy.optimize import minimize_scalar

    XJ, yJ = _mle_case(seed)
    g, lo, hi = 1e-4, 1e-3, 10.0
    t, it, flags = orc.mle_fit(XJ, yJ, g, 0.1, lo, hi, 1e-10, 200)
    grid = np.exp(np.linspace(np.log(lo), np.log(hi), 400))
    vals = [_np_loglik(XJ, yJ, g, th) for th in grid]
    i = int(np.argmax(vals))
    a, b = grid[max(i - 1, 0)], grid[min(i + 1, len(grid) - 1)]
    r = minimize_scalar(lambda u: -_np_loglik(XJ, yJ, g, np.exp(u)), bounds=(np.log(a), np.log(b)),
                        method="bounded", options={"xatol": 1e-12})
    tstar = float(np.exp(r.x))
    assert flags == 0 and it < 60
    assert t == pytest.approx(tstar, rel=1e-6)


def test_mle_fit_reports_a_bound(orc):
    """A response that is nearly linear across the design prefers the
    longest lengthscale: the estimate sits at dmax and says so."""
    rng = np.random.default_rng(48)
    XJ = rng.random((20, 2)) * 0.1
    yJ = 0.3 * XJ[:, 0] - 0.2 * XJ[:, 1] + 1.0
    t, it, flags = orc.mle_fit(XJ, yJ, 1e-4, 0.05, 1e-3, 0.5, 1e-8, 100)
    assert flags & orc.STATUS_MLE_BOUND
    assert t == pytest.approx(0.5, rel=1e-6)


def test_two_stage_is_search_estimate_search_estimate(orc):
    """Mode 2 = the design searched under the mode-1 estimate (the oracle's
    ordinary search with d = that estimate), the estimate refitted from it,
    and the GP prediction at the final estimate on the second design."""
    w = W.tiny_2d(M=3)
    prm = w.params.replace(scoring=W.SCORING_CHOL)
    o1 = orc.predict_mle(w.X, w.y, w.XX, prm, 1, nthreads=1)
    o2 = orc.predict_mle(w.X, w.y, w.XX, prm, 2, nthreads=1)
    g = prm.g
    for m in range(3):
        s2 = orc.predict(w.X, w.y, w.XX[m:m + 1], prm.replace(d=(float(o1["dhat"][m]),)), nthreads=1)
        assert np.array_equal(s2["sel"][0], o2["sel"][m])
        J = o2["sel"][m]
        t, _, _ = orc.mle_fit(w.X[J], w.y[J], g, float(o1["dhat"][m]), prm.d[0] / 1000, 100 * prm.d[0])
        assert t == o2["dhat"][m]
        # the prediction at the final estimate, against 40-digit arithmetic
        mp.mp.dps = 40
        th = mp.mpf(float(o2["dhat"][m]))
        P = [[mp.mpf(float(v)) for v in w.X[r]] for r in J]
        xm = [mp.mpf(float(v)) for v in w.XX[m]]
        kk = lambda a, b: mp.exp(-sum((ai - bi) ** 2 for ai, bi in zip(a, b)) / th)  # noqa: E731
        n = len(J)
        K = mp.matrix(n, n)
        for i in range(n):
            for k in range(n):
                K[i, k] = kk(P[i], P[k]) + (mp.mpf(g) if i == k else 0)
        kx = mp.matrix([kk(P[i], xm) for i in range(n)])
        yJ = mp.matrix([mp.mpf(float(w.y[r])) for r in J])
        a1, a2 = mp.lu_solve(K, kx), mp.lu_solve(K, yJ)
        mu = float(sum(a1[i] * yJ[i] for i in range(n)))
        s2 = float(sum(yJ[i] * a2[i] for i in range(n)) * (1 + mp.mpf(g) - sum(kx[i] * a1[i] for i in range(n))) / n)
        assert abs(o2["mean"][m] - mu) <= 1e-9 * abs(mu)
        assert abs(o2["s2"][m] - s2) <= 1e-7 * s2
    # the mode-1 design is the ordinary search under d0
    base = orc.predict(w.X, w.y, w.XX, prm, nthreads=1)
    assert np.array_equal(base["sel"], o1["sel"])


@pytest.mark.parametrize("search,numrays", [(W.SEARCH_RAY, 1), (W.SEARCH_NN, 0)])
def test_two_stage_with_rays_and_nearest_neighbours(orc, search, numrays):
    """Sec. 5 couples every design search with local inference.  With rays
    or nearest neighbours the stages compose the same way: the design
    searched under d0, the estimate fitted on it from d0, the design searched
    under that estimate, the estimate refitted from it.  The nearest-neighbour
    design is the n nearest by brute force at both stages (it does not depend
    on d), so its two stages share one design."""
    w = W.tiny_2d(M=3)
    prm = w.params.replace(search=search, numrays=numrays)
    o1 = orc.predict_mle(w.X, w.y, w.XX, prm, 1, nthreads=1)
    o2 = orc.predict_mle(w.X, w.y, w.XX, prm, 2, nthreads=1)
    lo, hi = prm.d[0] / 1000, 100 * prm.d[0]
    for m in range(3):
        s1 = orc.predict(w.X, w.y, w.XX[m:m + 1], prm, nthreads=1)["sel"][0]
        assert np.array_equal(s1, o1["sel"][m])
        t1, it1, _ = orc.mle_fit(w.X[s1], w.y[s1], prm.g, prm.d[0], lo, hi)
        assert t1 == o1["dhat"][m] and it1 == o1["iters"][m]
        s2 = orc.predict(w.X, w.y, w.XX[m:m + 1], prm.replace(d=(float(t1),)), nthreads=1)["sel"][0]
        assert np.array_equal(s2, o2["sel"][m])
        t2, it2, _ = orc.mle_fit(w.X[s2], w.y[s2], prm.g, t1, lo, hi)
        assert t2 == o2["dhat"][m] and it1 + it2 == o2["iters"][m]
        if search == W.SEARCH_NN:
            near = np.argsort(((w.X - w.XX[m]) ** 2).sum(axis=1), kind="stable")[:prm.n]
            assert set(near) == set(s1) == set(s2)
    assert np.all(np.isfinite(o2["mean"])) and np.all(o2["s2"] > 0)


# ------------------------------------------- global separable fit (O9) ---

def _np_sep_loglik(XS, yS, g, theta):
    D = (XS[:, None, :] - XS[None, :, :]) ** 2
    K = np.exp(-(D / np.asarray(theta)).sum(axis=2)) + g * np.eye(len(yS))
    _, logdet = np.linalg.slogdet(K)
    psi = yS @ np.linalg.solve(K, yS)
    return -0.5 * logdet - 0.5 * len(yS) * np.log(psi)


def _sep_case(seed, n=40, p=3):
    rng = np.random.default_rng(seed)
    XS = rng.random((n, p))
    yS = np.sin(3.0 * XS[:, 0]) + 0.5 * XS[:, 1] ** 2 + (0.1 * XS[:, 2] if p > 2 else 0.0)
    return XS, yS


@pytest.mark.parametrize("seed", [61, 62])
def test_sep_loglik_matches_numpy(orc, seed):
    XS, yS = _sep_case(seed)
    for theta in ([0.3, 1.0, 5.0], [0.05, 0.2, 0.7]):
        l, _, _ = orc.sep_eval(XS, yS, 1e-4, theta, 0)
        assert l == pytest.approx(_np_sep_loglik(XS, yS, 1e-4, theta), rel=1e-9, abs=1e-9)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_sep_derivatives_match_finite_differences(orc, k):
    """dl/dtheta_k against central differences of numpy's log-likelihood,
    d2l/dtheta_k^2 against central differences of the oracle's own first
    derivative (a dropped term, a wrong sign or the wrong coordinate fails)."""
    XS, yS = _sep_case(63)
    g = 1e-4
    theta = np.array([0.3, 1.0, 2.0])
    h = 1e-5 * theta[k]
    l, d1, d2 = orc.sep_eval(XS, yS, g, theta, k)
    tp, tm = theta.copy(), theta.copy()
    tp[k] += h
    tm[k] -= h
    fd1 = (_np_sep_loglik(XS, yS, g, tp) - _np_sep_loglik(XS, yS, g, tm)) / (2 * h)
    assert d1 == pytest.approx(fd1, rel=1e-5, abs=1e-6 * abs(l) / theta[k])
    fd2 = (orc.sep_eval(XS, yS, g, tp, k)[1] - orc.sep_eval(XS, yS, g, tm, k)[1]) / (2 * h)
    assert d2 == pytest.approx(fd2, rel=1e-5, abs=1e-6 * abs(d1) / theta[k] + 1e-3)


def test_sep_fit_with_one_input_is_the_isotropic_fit(orc):
    """p = 1: the separable exponent and derivatives are the isotropic ones,
    so the sweeps reach the isotropic estimate (to the Newton tolerance)."""
    XS, yS = _mle_case(44, n=30, p=1)
    t_iso, _, _ = orc.mle_fit(XS, yS, 1e-4, 0.1, 1e-3, 10.0, 1e-10, 200)
    th, it, fl = orc.sep_fit(XS, yS, 1e-4, 0.1, 1e-3, 10.0, 1e-10, 200, 10)
    assert fl == 0 and it > 1
    assert th[0] == pytest.approx(t_iso, rel=1e-8)


def test_sep_fit_is_a_maximiser(orc):
    """An interior estimate is a stationary point of numpy's likelihood in
    every coordinate, no worse than scipy's L-BFGS-B from the same start, and
    not improved by perturbing any coordinate."""
    from scipy.optimize import minimize

    XS, yS = _sep_case(64, n=50, p=2)
    g, lo, hi = 1e-4, 1e-3, 50.0
    th, it, fl = orc.sep_fit(XS, yS, g, 0.5, lo, hi, 1e-10, 200, 50)
    assert fl == 0
    l0 = _np_sep_loglik(XS, yS, g, th)
    for k in range(2):
        _, d1, d2 = orc.sep_eval(XS, yS, g, th, k)
        assert abs(d1) * th[k] <= 1e-6 * abs(l0) and d2 < 0
        for f in (1 - 1e-3, 1 + 1e-3):
            tq = th.copy()
            tq[k] *= f
            assert _np_sep_loglik(XS, yS, g, tq) < l0
    r = minimize(lambda u: -_np_sep_loglik(XS, yS, g, np.exp(u)), np.log([0.5, 0.5]), method="L-BFGS-B",
                 bounds=[(np.log(lo), np.log(hi))] * 2)
    assert l0 >= -r.fun - 1e-7 * abs(l0)


def test_sep_fit_sends_an_inert_input_to_the_upper_bound(orc):
    """A response that ignores an input prefers an unbounded lengthscale for
    it: the estimate sits at dmax and the status says so."""
    rng = np.random.default_rng(65)
    XS = rng.random((40, 2))
    yS = np.sin(4.0 * XS[:, 0])
    th, _, fl = orc.sep_fit(XS, yS, 1e-4, 0.5, 1e-3, 20.0, 1e-8, 100, 20)
    assert fl & orc.STATUS_MLE_BOUND
    assert th[1] == pytest.approx(20.0, rel=1e-6) and th[0] < 5.0
