"""Seeded synthetic workloads for local approximate GP prediction.

This module only draws inputs: design X (N x p), responses y (N), predictive
set XX (M x p) and the fixed method parameters of each workload.  It holds
none of the method's arithmetic, so both the CPU oracle and the HIP path read
the very same arrays from here.

The paper's own data (borehole, LGBB, Zhou, piston) are not reproduced; the
workloads below are synthetic stand-ins with the shapes the paper uses in its
experiments (Sec. 5: p = 2 and p = 8, N up to 1e6, n = 50, N' = 1000 nearest
candidates, a predictive set of 1e4 locations).

Seeds: numpy ``default_rng(14090074 + 100 * cfg + stream)`` with stream 0 for
the design, 1 for the predictive set and 2 for request arrivals.  The ray
workload reuses the design and predictive set of the exhaustive 8-d one.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 14090074

SEARCH_EXHAUSTIVE = 0
SEARCH_RAY = 1
SEARCH_NN = 2

PREC_FP64 = 0
PREC_MIXED = 1

SCORING_PARTINV = 0
SCORING_CHOL = 1
SNAP_CANDIDATES = 0  # ray search: snap to the nearest of the N' candidates
SNAP_DESIGN = 1      # ray search: snap to the nearest of the whole design (Sec. 5)


@dataclasses.dataclass
class Params:
    """Method knobs, laGP-style (Sec. 2.2 and Sec. 5 of the paper).

    n0: size of the nearest-neighbour starting design; n: final local design
    size; ncand: N', the number of nearest candidates searched; search: one of
    SEARCH_*; numrays: rays per greedy step (ray search); d: lengthscale(s),
    one value (isotropic) or p values (separable); g: nugget; precision:
    PREC_FP64 or PREC_MIXED; rescore_k: FP64 re-scored shortlist in the mixed
    form; brent_maxit / brent_tol: the line-search budget and tolerance;
    scoring: SCORING_PARTINV (partitioned-inverse updates) or SCORING_CHOL
    (incremental Cholesky columns) for exhaustive search; snap: SNAP_CANDIDATES
    or SNAP_DESIGN, where ray search snaps its optimum to.
    """

    n0: int = 6
    n: int = 50
    ncand: int = 1000
    search: int = SEARCH_EXHAUSTIVE
    numrays: int = 0
    d: tuple = (0.1,)
    g: float = 1e-6
    precision: int = PREC_FP64
    rescore_k: int = 16
    brent_maxit: int = 100
    brent_tol: float = 2.0 ** -13
    scoring: int = SCORING_PARTINV
    snap: int = SNAP_CANDIDATES

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class Workload:
    name: str
    X: np.ndarray
    y: np.ndarray
    XX: np.ndarray
    params: Params
    truth: np.ndarray | None = None  # noise-free response at XX, for RMSE


def _rng(cfg: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + 100 * cfg + stream)


def f_bump2(X: np.ndarray) -> np.ndarray:
    """2-d response: exp(-((x1-.5)^2+(x2-.5)^2)/0.08) sin(6 x1) + 0.3 cos(5 x2)."""
    x1, x2 = X[:, 0], X[:, 1]
    return np.exp(-((x1 - 0.5) ** 2 + (x2 - 0.5) ** 2) / 0.08) * np.sin(6.0 * x1) + 0.3 * np.cos(5.0 * x2)


def f_sines8(X: np.ndarray) -> np.ndarray:
    """8-d response: sum_j sin(2 pi w_j x_j) + x1 x2 x3, w_j = 0.5 + 0.25 j."""
    w = 0.5 + 0.25 * np.arange(1, X.shape[1] + 1)
    return np.sin(2.0 * math.pi * w[None, :] * X).sum(axis=1) + X[:, 0] * X[:, 1] * X[:, 2]


def f_mix4(X: np.ndarray) -> np.ndarray:
    """4-d response: sin(3 x1) cos(2 x2) + x3^2 - 0.5 x4."""
    return np.sin(3.0 * X[:, 0]) * np.cos(2.0 * X[:, 1]) + X[:, 2] ** 2 - 0.5 * X[:, 3]


def w_sec51(x: np.ndarray) -> np.ndarray:
    """The factor of the 2-d test function of Sec. 5.1:
    w(x) = exp(-(x-1)^2) + exp(-0.8 (x+1)^2) - 0.05 sin(8 (x+0.1))."""
    return np.exp(-((x - 1.0) ** 2)) + np.exp(-0.8 * (x + 1.0) ** 2) - 0.05 * np.sin(8.0 * (x + 0.1))


def f_sec51(X: np.ndarray) -> np.ndarray:
    """The 2-d test function of Sec. 5.1: f(x1, x2) = -w(x1) w(x2)."""
    return -w_sec51(X[:, 0]) * w_sec51(X[:, 1])


def f_aniso8(X: np.ndarray) -> np.ndarray:
    """Anisotropic 8-d response: sin(3 pi x1) + 2 x2^2 - x3 + 0.2 sin(2 pi x4);
    x5..x8 do not enter (global lengthscales differ by orders of magnitude
    across the inputs)."""
    return (np.sin(3.0 * math.pi * X[:, 0]) + 2.0 * X[:, 1] ** 2 - X[:, 2]
            + 0.2 * np.sin(2.0 * math.pi * X[:, 3]))


def grid2(side: int) -> np.ndarray:
    """Regular side x side grid on [0,1]^2, x = i/(side-1); first axis slowest."""
    g = np.arange(side, dtype=np.float64) / (side - 1)
    a, b = np.meshgrid(g, g, indexing="ij")
    return np.ascontiguousarray(np.stack([a.ravel(), b.ravel()], axis=1))


def tiny_2d(M: int | None = None) -> Workload:
    """N = 4000 iid uniform design on [0,1]^2, 100 uniform predictive locations,
    d = 0.1, g = 1e-6, n0 = 6, n = 50, exhaustive over the 500 nearest."""
    X = _rng(0, 0).random((4000, 2))
    XX = _rng(0, 1).random((100, 2))
    if M is not None:
        XX = XX[:M]
    p = Params(n0=6, n=50, ncand=500, search=SEARCH_EXHAUSTIVE, d=(0.1,), g=1e-6)
    return Workload("uniform2d_N4000_M100_n50_cand500_exhaustive", X, f_bump2(X), XX, p, f_bump2(XX))


def uniform8d(M: int | None = None, N: int = 1_000_000, search: int = SEARCH_EXHAUSTIVE) -> Workload:
    """N = 1e6 iid uniform design on [0,1]^8, 1e4 uniform predictive locations,
    separable kernel with d_k = 0.5 in every dimension, g = 1e-6, n0 = 6,
    n = 50, 1000 nearest candidates; exhaustive, or 10 rays per step."""
    X = _rng(1, 0).random((N, 8))
    XX = _rng(1, 1).random((10_000, 8))
    if M is not None:
        XX = XX[:M]
    p = Params(n0=6, n=50, ncand=1000, search=search, numrays=10 if search == SEARCH_RAY else 0,
               d=(0.5,) * 8, g=1e-6)
    mode = {SEARCH_EXHAUSTIVE: "exhaustive", SEARCH_RAY: "ray10", SEARCH_NN: "nn"}[search]
    return Workload(f"uniform8d_N{N}_M{XX.shape[0]}_n50_cand1000_{mode}", X, f_sines8(X), XX, p, f_sines8(XX))


def grid2d(M: int | None = None, side: int = 1000, precision: int = PREC_FP64) -> Workload:
    """1000 x 1000 grid design on [0,1]^2 with the 2-d bump response, 1e5
    uniform predictive locations, 4000 nearest candidates, n = 100,
    d = 0.05, g = 1e-6, n0 = 6, exhaustive; FP64 or mixed precision."""
    X = grid2(side)
    XX = _rng(3, 1).random((100_000, 2))
    if M is not None:
        XX = XX[:M]
    p = Params(n0=6, n=100, ncand=4000, search=SEARCH_EXHAUSTIVE, d=(0.05,), g=1e-6, precision=precision)
    tag = "mixed" if precision == PREC_MIXED else "fp64"
    return Workload(f"grid2d_N{side * side}_M{XX.shape[0]}_n100_cand4000_{tag}", X, f_bump2(X), XX, p, f_bump2(XX))


def paper2d(M: int | None = None, n: int = 50, search: int = SEARCH_EXHAUSTIVE, numrays: int = 1,
            ncand: int = 1000, scoring: int = SCORING_CHOL) -> Workload:
    """The 2-d experiment of Sec. 5.1: a 201 x 201 grid design on [-2, 2]^2
    (N = 40401, spacing 0.02) with f = -w(x1) w(x2), no noise, and a 99 x 99
    predictive grid spaced to avoid the design: x_i = -1.95 + 0.04 i in each
    coordinate (every value midway between two design lines).  n0 = 6,
    N' = 1000 nearest candidates, one ray per step (as the section uses on
    this dense design), starting lengthscale d0 = 0.5 (the value of the
    section's illustrations on this grid; it is refitted by local MLE) and
    nugget g = 1e-6."""
    t = -2.0 + 0.02 * np.arange(201, dtype=np.float64)
    a, b = np.meshgrid(t, t, indexing="ij")
    X = np.ascontiguousarray(np.stack([a.ravel(), b.ravel()], axis=1))
    u = -1.95 + 0.04 * np.arange(99, dtype=np.float64)
    a, b = np.meshgrid(u, u, indexing="ij")
    XX = np.ascontiguousarray(np.stack([a.ravel(), b.ravel()], axis=1))
    if M is not None:
        XX = XX[:M]
    ray = search == SEARCH_RAY
    p = Params(n0=6, n=n, ncand=ncand, search=search, numrays=numrays if ray else 0, d=(0.5,), g=1e-6,
               scoring=scoring if search == SEARCH_EXHAUSTIVE else SCORING_PARTINV)
    mode = {SEARCH_EXHAUSTIVE: "exhaustive", SEARCH_RAY: f"ray{numrays}", SEARCH_NN: "nn"}[search]
    return Workload(f"sec51grid2d_N40401_M{XX.shape[0]}_n{n}_cand{ncand}_{mode}", X, f_sec51(X), XX, p,
                    f_sec51(XX))


def aniso8d(M: int | None = None, N: int = 1_000_000) -> Workload:
    """N = 1e6 iid uniform design on [0,1]^8 with the anisotropic response,
    1e4 uniform predictive locations, isotropic d0 = 0.5 (refitted by local
    MLE), g = 1e-6, n0 = 6, n = 50, 1000 nearest candidates.  Pre-scaling
    fits global separable lengthscales on the subset ``aniso8d_subset``."""
    X = _rng(5, 0).random((N, 8))
    XX = _rng(5, 1).random((10_000, 8))
    if M is not None:
        XX = XX[:M]
    p = Params(n0=6, n=50, ncand=1000, d=(0.5,), g=1e-6, scoring=SCORING_CHOL)
    return Workload(f"aniso8d_N{N}_M{XX.shape[0]}_n50_cand1000", X, f_aniso8(X), XX, p, f_aniso8(XX))


def aniso8d_subset(N: int, ns: int = 256) -> np.ndarray:
    """Rows of the global fit's subset: ns distinct rows drawn uniformly."""
    return np.sort(_rng(5, 3).choice(N, size=ns, replace=False))


def serving4d(N: int = 2_000_000) -> Workload:
    """Resident serving design: N = 2e6 iid uniform on [0,1]^4 with the 4-d
    response; d = 0.1, g = 1e-6, n0 = 6, 4 rays, 1000 nearest candidates.
    Requests are drawn by ``serving_requests``; XX here is empty."""
    X = _rng(4, 0).random((N, 4))
    p = Params(n0=6, n=50, ncand=1000, search=SEARCH_EXHAUSTIVE, numrays=4, d=(0.1,), g=1e-6)
    return Workload(f"uniform4d_N{N}_serving", X, f_mix4(X), np.zeros((0, 4)), p, None)


@dataclasses.dataclass
class Request:
    arrival_s: float
    XX: np.ndarray
    n: int
    search: int
    precision: int


def serving_requests(count: int, qps: float, precision_mix: float = 0.0, p: int = 4) -> list[Request]:
    """Open-loop Poisson arrivals at rate ``qps``; each request carries
    floor(10**U(0,3)) locations (1..1000, log-uniform), n from {30, 50, 100},
    exhaustive or ray search at 50/50, and an exhaustive request in the
    mixed form with probability ``precision_mix`` (the mixed screen scores
    exhaustive searches only)."""
    rng = _rng(4, 2)
    t = 0.0
    out = []
    for _ in range(count):
        t += rng.exponential(1.0 / qps)
        m = int(np.floor(10.0 ** rng.uniform(0.0, 3.0)))
        m = max(1, min(1000, m))
        XX = rng.random((m, p))
        n = int(rng.choice([30, 50, 100]))
        search = SEARCH_RAY if rng.random() < 0.5 else SEARCH_EXHAUSTIVE
        mixed = rng.random() < precision_mix
        prec = PREC_MIXED if mixed and search == SEARCH_EXHAUSTIVE else PREC_FP64
        out.append(Request(t, XX, n, search, prec))
    return out


def ray_candidates_needed(n: int, n0: int, numrays: int) -> int:
    """Candidates a ray search's starts reach (Sec. 4): at step j the starts
    are the remaining ranks k .. k + R - 1 with j taken, k = t mod
    floor(sqrt t), t = j - n0 + 1; so n - 1 + R + the largest such k."""
    off = 0
    for t in range(1, n - n0 + 1):
        r = math.isqrt(t)
        off = max(off, t % r if r else 0)
    return n - 1 + numrays + off


def small_case(seed: int, N: int, p: int, M: int, **kw) -> Workload:
    """Small uniform workloads for parity sweeps: design and locations iid
    uniform on [0,1]^p, the 2-d bump response (p = 2) or the 8-d sines
    response restricted to p dims otherwise."""
    rng = np.random.default_rng(SEED_BASE + 7919 * seed)
    X = rng.random((N, p))
    XX = rng.random((M, p))
    if p == 2:
        y = f_bump2(X)
    else:
        y = f_sines8(np.pad(X, ((0, 0), (0, max(0, 3 - p))))) if p < 3 else f_sines8(X)
    params = Params(**kw)
    return Workload(f"small_s{seed}_N{N}_p{p}_M{M}", X, y, XX, params, None)


WORKLOADS = {
    "uniform2d_tiny": tiny_2d,
    "uniform8d_exhaustive": lambda M=None: uniform8d(M, search=SEARCH_EXHAUSTIVE),
    "uniform8d_ray": lambda M=None: uniform8d(M, search=SEARCH_RAY),
    "sec51grid2d": paper2d,
    "grid2d_fp64": lambda M=None: grid2d(M, precision=PREC_FP64),
    "grid2d_mixed": lambda M=None: grid2d(M, precision=PREC_MIXED),
}
