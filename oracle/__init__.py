"""ctypes loader for the plain FP64 CPU oracle (``lagp_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product path never does.
It shares no code with the HIP library and imports nothing from it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lagp_oracle.c")
LIB = os.path.join(HERE, "liblagp_oracle.so")
NDIAG = 8

STATUS_VNONPOS = 1
STATUS_NONFINITE = 2
STATUS_NOTPD = 4
STATUS_BADRAY = 8
STATUS_MLE_BOUND = 16
STATUS_MLE_NOTPD = 32
STATUS_MLE_MAXIT = 64

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
BRENT_FN = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.c_double, ctypes.c_void_p)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        L.orc_knn.argtypes = [_dp, ctypes.c_int64, ctypes.c_int, _dp, ctypes.c_int64, ctypes.c_int, _i64p, _dp,
                              ctypes.c_int]
        L.orc_knn.restype = ctypes.c_int
        common = [_dp, _dp, ctypes.c_int64, ctypes.c_int]
        par = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int,
               ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int]
        L.orc_predict.argtypes = common + [_dp, ctypes.c_int64] + par + [_i32p, ctypes.c_int, _dp, _dp, _dp, _i32p,
                                                                          _dp, _i32p]
        L.orc_predict.restype = ctypes.c_int
        L.orc_trace.argtypes = common + [_dp] + par + [_i32p, _dp, _dp, _dp, _i32p, _dp, _dp, _dp, _i64p]
        L.orc_trace.restype = ctypes.c_int
        L.orc_brent_min.argtypes = [BRENT_FN, ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int, ctypes.POINTER(ctypes.c_int), _dp, _dp]
        L.orc_brent_min.restype = ctypes.c_double
        L.orc_ray_k0.argtypes = [ctypes.c_int]
        L.orc_ray_k0.restype = ctypes.c_int
        L.orc_ray_segment.argtypes = [_dp, _dp, _dp, _dp, ctypes.c_int, _dp]
        L.orc_ray_segment.restype = ctypes.c_double
        L.orc_exp.argtypes = [ctypes.c_double]
        L.orc_exp.restype = ctypes.c_double
        L.orc_kern.argtypes = [_dp, _dp, ctypes.c_int, _dp, ctypes.c_int]
        L.orc_kern.restype = ctypes.c_double
        L.orc_sqdist.argtypes = [_dp, _dp, ctypes.c_int]
        L.orc_sqdist.restype = ctypes.c_double
        L.orc_spd_inverse.argtypes = [_dp, ctypes.c_int, _dp]
        L.orc_spd_inverse.restype = ctypes.c_int
        i32 = ctypes.c_int
        L.orc_predict_mle.argtypes = common + [_dp, ctypes.c_int64, i32, i32, i32, i32, i32, ctypes.c_double,
                                               ctypes.c_double, i32, ctypes.c_double, i32, i32, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_double, i32, i32,
                                               _dp, _dp, _dp, _i32p, _dp, _i32p, _i32p]
        L.orc_predict_mle.restype = ctypes.c_int
        L.orc_mle_eval.argtypes = [i32, i32, _dp, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.orc_mle_eval.restype = ctypes.c_int
        L.orc_mle_fit.argtypes = [i32, i32, _dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.orc_mle_fit.restype = ctypes.c_double
        L.orc_sep_eval.argtypes = [i32, i32, _dp, _dp, ctypes.c_double, _dp, i32, _dp]
        L.orc_sep_eval.restype = ctypes.c_int
        L.orc_sep_fit.argtypes = [i32, i32, _dp, _dp, ctypes.c_double, _dp, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, i32, i32, ctypes.POINTER(i32)]
        L.orc_sep_fit.restype = ctypes.c_int
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


def default_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def knn(X, XX, ncand: int, nthreads: int | None = None):
    """Nearest ``ncand`` design rows for each row of XX: (idx int64, d2)."""
    X, XX = _f64(X), _f64(np.atleast_2d(XX))
    N, p = X.shape
    M = XX.shape[0]
    idx = np.empty((M, ncand), np.int64)
    d2 = np.empty((M, ncand), np.float64)
    rc = lib().orc_knn(_p(X), N, p, _p(XX), M, ncand, _p(idx, _i64p), _p(d2), nthreads or default_threads())
    if rc != 0:
        raise ValueError(f"orc_knn failed: {rc}")
    return idx, d2


def _ncand(params, N):
    """N' as the search sees it: a ray search that snaps over the whole design
    (Sec. 5 places no N' limit on ray searches) is the same search with every
    design row a candidate, nearest first."""
    return N if getattr(params, "snap", 0) == 1 else params.ncand


def _par(params, p, N):
    d = _f64(np.atleast_1d(params.d))
    return d, [params.n0, params.n, _ncand(params, N), params.search, params.numrays, _p(d), len(d), params.g,
               params.brent_maxit, params.brent_tol, getattr(params, "scoring", 0)]


def predict(X, y, XX, params, forced=None, nthreads: int | None = None):
    """Local GP prediction at every row of XX.  ``forced`` (M x n row ids)
    replays a given selection sequence; the per-step diagnostics then hold the
    oracle's own choice beside the forced one."""
    X, y, XX = _f64(X), _f64(y), _f64(np.atleast_2d(XX))
    N, p = X.shape
    M = XX.shape[0]
    n, n0 = params.n, params.n0
    nd = 0 if params.search == 2 else n - n0
    d, par = _par(params, p, N)
    out = dict(mean=np.empty(M), s2=np.empty(M), df=np.empty(M), sel=np.empty((M, n), np.int32),
               diag=np.empty((M, nd, NDIAG)), status=np.empty(M, np.int32))
    fz = None if forced is None else np.ascontiguousarray(forced, dtype=np.int32)
    rc = lib().orc_predict(_p(X), _p(y), N, p, _p(XX), M, *par, _p(fz, _i32p), nthreads or default_threads(),
                           _p(out["mean"]), _p(out["s2"]), _p(out["df"]), _p(out["sel"], _i32p), _p(out["diag"]),
                           _p(out["status"], _i32p))
    if rc != 0:
        raise ValueError(f"orc_predict failed: {rc}")
    return out


def trace(X, y, x, params, forced=None):
    """One location with full traces: ALC of every candidate at every step,
    the final inverse and the candidate list (for brute-force checks)."""
    X, y, x = _f64(X), _f64(y), _f64(np.ravel(x))
    N, p = X.shape
    n, n0, nc = params.n, params.n0, _ncand(params, N)
    nd = 0 if params.search == 2 else n - n0
    d, par = _par(params, p, N)
    mean, s2, df = (ctypes.c_double(), ctypes.c_double(), ctypes.c_double())
    out = dict(sel=np.empty(n, np.int32), diag=np.empty((nd, NDIAG)), alc=np.empty((nd, nc)),
               Ki=np.empty((n, n)), cand=np.empty(nc, np.int64))
    fz = None if forced is None else np.ascontiguousarray(forced, dtype=np.int32)
    st = lib().orc_trace(_p(X), _p(y), N, p, _p(x), *par, _p(fz, _i32p), ctypes.byref(mean), ctypes.byref(s2),
                         ctypes.byref(df), _p(out["sel"], _i32p), _p(out["diag"]), _p(out["alc"]), _p(out["Ki"]),
                         _p(out["cand"], _i64p))
    if st < 0:
        raise ValueError(f"orc_trace failed: {st}")
    out.update(mean=mean.value, s2=s2.value, df=df.value, status=st)
    return out


def predict_mle(X, y, XX, params, mode: int, dmin: float = 0.0, dmax: float = 0.0, tol: float = 0.0,
                maxit: int = 0, nthreads: int | None = None):
    """Local MLE of an isotropic lengthscale (mode 1: on the design searched
    under params.d; mode 2: two-stage re-design) and the prediction under the
    estimate, at every row of XX (any search mode of params; exhaustive
    search scored as params.scoring)."""
    X, y, XX = _f64(X), _f64(y), _f64(np.atleast_2d(XX))
    N, p = X.shape
    M = XX.shape[0]
    n = params.n
    d0 = float(np.atleast_1d(params.d)[0])
    out = dict(mean=np.empty(M), s2=np.empty(M), df=np.empty(M), sel=np.empty((M, n), np.int32),
               dhat=np.empty(M), iters=np.empty(M, np.int32), status=np.empty(M, np.int32))
    rc = lib().orc_predict_mle(_p(X), _p(y), N, p, _p(XX), M, params.n0, n, _ncand(params, N), params.search,
                               params.numrays, d0, params.g, params.brent_maxit, params.brent_tol,
                               getattr(params, "scoring", 0), mode, dmin, dmax, tol, maxit,
                               nthreads or default_threads(), _p(out["mean"]), _p(out["s2"]), _p(out["df"]),
                               _p(out["sel"], _i32p), _p(out["dhat"]), _p(out["iters"], _i32p),
                               _p(out["status"], _i32p))
    if rc != 0:
        raise ValueError(f"orc_predict_mle failed: {rc}")
    return out


def mle_eval(XJ, yJ, g: float, theta: float):
    """(l, l', l'') of the local likelihood at theta, or None if K is not
    positive definite."""
    XJ, yJ = _f64(XJ), _f64(yJ)
    out = np.empty(3)
    rc = lib().orc_mle_eval(XJ.shape[0], XJ.shape[1], _p(XJ), _p(yJ), g, theta, _p(out))
    return None if rc != 0 else tuple(out)


def mle_fit(XJ, yJ, g: float, theta0: float, dmin: float, dmax: float, tol: float = 1e-8, maxit: int = 100):
    """(theta_hat, evaluations, flags) of the safeguarded Newton maximisation."""
    XJ, yJ = _f64(XJ), _f64(yJ)
    it, fl = ctypes.c_int(), ctypes.c_int()
    t = lib().orc_mle_fit(XJ.shape[0], XJ.shape[1], _p(XJ), _p(yJ), g, theta0, dmin, dmax, tol, maxit,
                          ctypes.byref(it), ctypes.byref(fl))
    return t, it.value, fl.value


def sep_eval(XS, yS, g: float, theta, k: int):
    """(l, dl/dtheta_k, d2l/dtheta_k^2) of the separable likelihood, or None
    if K is not positive definite."""
    XS, yS = _f64(XS), _f64(yS)
    th = _f64(np.atleast_1d(theta)).copy()
    out = np.empty(3)
    rc = lib().orc_sep_eval(XS.shape[0], XS.shape[1], _p(XS), _p(yS), g, _p(th), int(k), _p(out))
    if rc == -2:
        raise ValueError("orc_sep_eval: bad arguments")
    return None if rc != 0 else tuple(out)


def sep_fit(XS, yS, g: float, theta0, dmin: float, dmax: float, tol: float = 1e-8, maxit: int = 100,
            maxsweep: int = 20):
    """Global separable lengthscales by coordinate-wise Newton sweeps:
    (theta_hat (p,), evaluations, flags)."""
    XS, yS = _f64(XS), _f64(yS)
    th = _f64(np.broadcast_to(np.atleast_1d(theta0), (XS.shape[1],))).copy()
    it = ctypes.c_int()
    fl = lib().orc_sep_fit(XS.shape[0], XS.shape[1], _p(XS), _p(yS), g, _p(th), dmin, dmax, tol, maxit, maxsweep,
                           ctypes.byref(it))
    if fl < 0:
        raise ValueError(f"orc_sep_fit failed: {fl}")
    return th, it.value, fl


def brent_min(f, lo: float, hi: float, tol: float = 2.0 ** -13, maxit: int = 100):
    """Minimise f on [lo, hi]; returns (xmin, fmin, evaluations, min decision gap)."""
    cb = BRENT_FN(lambda t, _ctx: float(f(t)))
    ne = ctypes.c_int()
    gap = ctypes.c_double()
    fb = ctypes.c_double()
    x = lib().orc_brent_min(cb, None, lo, hi, tol, maxit, ctypes.byref(ne), ctypes.byref(gap), ctypes.byref(fb))
    return x, fb.value, ne.value, gap.value


def ray_k0(t: int) -> int:
    return lib().orc_ray_k0(int(t))


def ray_segment(a, x, lo, hi):
    a, x, lo, hi = _f64(a), _f64(x), _f64(lo), _f64(hi)
    d = np.empty_like(a)
    tau = lib().orc_ray_segment(_p(a), _p(x), _p(lo), _p(hi), a.size, _p(d))
    return tau, d


def exp(x: float) -> float:
    return lib().orc_exp(float(x))


def kern(a, b, d):
    a, b, d = _f64(a), _f64(b), _f64(np.atleast_1d(d))
    return lib().orc_kern(_p(a), _p(b), a.size, _p(d), d.size)


def sqdist(a, b):
    a, b = _f64(a), _f64(b)
    return lib().orc_sqdist(_p(a), _p(b), a.size)


def spd_inverse(A):
    A = _f64(A)
    out = np.empty_like(A)
    rc = lib().orc_spd_inverse(_p(A), A.shape[0], _p(out))
    if rc != 0:
        raise np.linalg.LinAlgError("not positive definite")
    return out
