"""MI355X local approximate GP prediction: Python binding of liblagp.so.

The functions below carry the names of the C ABI in include/lagp.h and only
marshal arguments: torch CUDA tensors (ROCm) in and out, the current torch
stream by default.  Every step of the computation runs in the HIP library;
if the library is missing this module raises instead of computing anything
itself.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import workloads  # noqa: F401  (seeded inputs; no method arithmetic)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblagp.so")

LAGP_OK = 0
LAGP_EINVAL = -1
LAGP_ENOMEM = -2
LAGP_EDEVICE = -3
LAGP_EAGAIN = -4
LAGP_WARN_NUMERIC = 1
LAGP_MAX_DIM = 16
LAGP_SEARCH_EXHAUSTIVE = 0
LAGP_SEARCH_RAY = 1
LAGP_SEARCH_NN = 2
LAGP_PREC_FP64 = 0
LAGP_PREC_MIXED = 1
LAGP_SCORING_PARTINV = 0
LAGP_SCORING_CHOL = 1
LAGP_STATUS_VNONPOS = 1
LAGP_STATUS_NONFINITE = 2
LAGP_STATUS_NOTPD = 4
LAGP_STATUS_MLE_BOUND = 16
LAGP_STATUS_MLE_NOTPD = 32
LAGP_STATUS_MLE_MAXIT = 64

EXPORTED = [
    "lagp_version", "lagp_last_error", "lagp_design_create", "lagp_design_destroy", "lagp_design_info",
    "lagp_design_build_grid",
    "lagp_candidates", "lagp_predict", "lagp_predict_candidates", "lagp_predict_counts", "lagp_predict_noalloc",
    "lagp_predict_mle",
    "lagp_fit_separable",
    "lagp_prescale", "lagp_server_create", "lagp_server_submit", "lagp_server_poll",
    "lagp_server_fetch", "lagp_server_stats", "lagp_server_destroy",
]


class lagp_params(ctypes.Structure):
    _fields_ = [
        ("n0", ctypes.c_int32), ("n", ctypes.c_int32), ("ncand", ctypes.c_int32), ("numrays", ctypes.c_int32),
        ("search", ctypes.c_int32), ("precision", ctypes.c_int32), ("d_len", ctypes.c_int32),
        ("rescore_k", ctypes.c_int32), ("d", ctypes.c_double * LAGP_MAX_DIM), ("g", ctypes.c_double),
        ("brent_maxit", ctypes.c_int32), ("scoring", ctypes.c_int32), ("brent_tol", ctypes.c_double),
        ("snap", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class lagp_mle_params(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("maxit", ctypes.c_int32), ("dmin", ctypes.c_double),
                ("dmax", ctypes.c_double), ("tol", ctypes.c_double)]


class LagpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"liblagp error {code}: {msg}")
        self.code = code


_lib = None
_vp = ctypes.c_void_p


def lib():
    """Load liblagp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1409_0074_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        pp = ctypes.POINTER(lagp_params)
        L.lagp_version.restype = i32
        L.lagp_last_error.restype = ctypes.c_char_p
        L.lagp_design_create.argtypes = [_vp, _vp, i64, i32, _vp, ctypes.POINTER(_vp)]
        L.lagp_design_create.restype = i32
        L.lagp_design_destroy.argtypes = [_vp]
        L.lagp_design_destroy.restype = None
        L.lagp_design_info.argtypes = [_vp, ctypes.POINTER(i64), ctypes.POINTER(i32)]
        L.lagp_design_info.restype = i32
        L.lagp_design_build_grid.argtypes = [_vp, _vp]
        L.lagp_design_build_grid.restype = i32
        L.lagp_candidates.argtypes = [_vp, _vp, i64, i32, _vp, _vp, _vp]
        L.lagp_candidates.restype = i32
        L.lagp_predict.argtypes = [_vp, _vp, i64, pp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.lagp_predict.restype = i32
        L.lagp_predict_candidates.argtypes = [_vp, _vp, i64, _vp, pp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.lagp_predict_candidates.restype = i32
        L.lagp_predict_counts.argtypes = [_vp, _vp, i64, _vp, pp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.lagp_predict_counts.restype = i32
        L.lagp_predict_noalloc.argtypes = [_vp, _vp, i64, pp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.lagp_predict_noalloc.restype = i32
        L.lagp_predict_mle.argtypes = [_vp, _vp, i64, _vp, pp, ctypes.POINTER(lagp_mle_params), _vp, _vp, _vp, _vp,
                                       _vp, _vp, _vp, _vp]
        L.lagp_predict_mle.restype = i32
        dp = ctypes.POINTER(ctypes.c_double)
        L.lagp_fit_separable.argtypes = [_vp, _vp, i32, i32, ctypes.c_double, dp, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), _vp]
        L.lagp_fit_separable.restype = i32
        L.lagp_prescale.argtypes = [_vp, i64, i32, dp, _vp, _vp]
        L.lagp_prescale.restype = i32
        L.lagp_server_create.argtypes = [_vp, sz, i32, ctypes.POINTER(_vp)]
        L.lagp_server_create.restype = i32
        L.lagp_server_submit.argtypes = [_vp, _vp, i64, pp, ctypes.POINTER(ctypes.c_uint64)]
        L.lagp_server_submit.restype = i32
        L.lagp_server_poll.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(i32)]
        L.lagp_server_poll.restype = i32
        L.lagp_server_fetch.argtypes = [_vp, ctypes.c_uint64, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double)]
        L.lagp_server_fetch.restype = i32
        L.lagp_server_stats.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double), i32]
        L.lagp_server_stats.restype = i32
        L.lagp_server_destroy.argtypes = [_vp]
        L.lagp_server_destroy.restype = None
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc < 0:
        raise LagpError(rc, lib().lagp_last_error().decode())
    return rc


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def make_params(params=None, **kw) -> lagp_params:
    """lagp_params from a workloads.Params (or keyword overrides)."""
    src = params if params is not None else workloads.Params()
    if kw:
        src = src.replace(**kw)
    P = lagp_params()
    P.n0, P.n, P.ncand = src.n0, src.n, src.ncand
    P.numrays, P.search, P.precision = src.numrays, src.search, src.precision
    d = np.atleast_1d(np.asarray(src.d, dtype=np.float64))
    P.d_len = int(d.size)
    for k, v in enumerate(d):
        P.d[k] = float(v)
    P.g = float(src.g)
    P.rescore_k = src.rescore_k
    P.brent_maxit = src.brent_maxit
    P.brent_tol = float(src.brent_tol)
    P.scoring = src.scoring
    P.snap = src.snap
    return P


# ---------------------------------------------------------------- C ABI --

def lagp_version() -> int:
    return lib().lagp_version()


def lagp_last_error() -> str:
    return lib().lagp_last_error().decode()


def lagp_design_create(X, y, stream=None):
    """Device copy of the design; X (N x p) and y (N) float64 tensors."""
    h = _vp()
    _check(lib().lagp_design_create(_ptr(X), _ptr(y), X.shape[0], X.shape[1], _stream(stream), ctypes.byref(h)))
    return h


def lagp_design_destroy(design) -> None:
    lib().lagp_design_destroy(design)


def lagp_design_build_grid(design, stream=None) -> int:
    return _check(lib().lagp_design_build_grid(design, _stream(stream)))


def lagp_design_info(design):
    N, p = ctypes.c_int64(), ctypes.c_int32()
    _check(lib().lagp_design_info(design, ctypes.byref(N), ctypes.byref(p)))
    return N.value, p.value


def lagp_candidates(design, XX, ncand, cand_idx, cand_d2=None, stream=None) -> int:
    return _check(lib().lagp_candidates(design, _ptr(XX), XX.shape[0], int(ncand), _ptr(cand_idx), _ptr(cand_d2),
                                        _stream(stream)))


def lagp_predict(design, XX, params: lagp_params, mean, s2, df, sel_idx=None, diag=None, status=None,
                 stream=None) -> int:
    return _check(lib().lagp_predict(design, _ptr(XX), XX.shape[0], ctypes.byref(params), _ptr(mean), _ptr(s2),
                                     _ptr(df), _ptr(sel_idx), _ptr(diag), _ptr(status), _stream(stream)))


def lagp_predict_candidates(design, XX, cand_idx, params: lagp_params, mean, s2, df, sel_idx=None, diag=None,
                            status=None, stream=None) -> int:
    return _check(lib().lagp_predict_candidates(design, _ptr(XX), XX.shape[0], _ptr(cand_idx), ctypes.byref(params),
                                                _ptr(mean), _ptr(s2), _ptr(df), _ptr(sel_idx), _ptr(diag),
                                                _ptr(status), _stream(stream)))


def lagp_predict_counts(design, XX, cand_idx, params: lagp_params, mean, s2, df, sel_idx=None, diag=None,
                        status=None, counts=None, stream=None) -> int:
    return _check(lib().lagp_predict_counts(design, _ptr(XX), XX.shape[0], _ptr(cand_idx), ctypes.byref(params),
                                            _ptr(mean), _ptr(s2), _ptr(df), _ptr(sel_idx), _ptr(diag),
                                            _ptr(status), _ptr(counts), _stream(stream)))


def lagp_predict_noalloc(design, XX, params: lagp_params, mean, s2, df, sel_idx=None, diag=None, status=None,
                         stream=None) -> int:
    return _check(lib().lagp_predict_noalloc(design, _ptr(XX), XX.shape[0], ctypes.byref(params), _ptr(mean),
                                             _ptr(s2), _ptr(df), _ptr(sel_idx), _ptr(diag), _ptr(status),
                                             _stream(stream)))


def make_mle_params(mode: int, dmin: float = 0.0, dmax: float = 0.0, tol: float = 0.0,
                    maxit: int = 0) -> lagp_mle_params:
    M = lagp_mle_params()
    M.mode, M.maxit, M.dmin, M.dmax, M.tol = int(mode), int(maxit), float(dmin), float(dmax), float(tol)
    return M


def lagp_predict_mle(design, XX, cand_idx, params: lagp_params, mle: lagp_mle_params, mean, s2, df, dhat,
                     sel_idx=None, iters=None, status=None, stream=None) -> int:
    return _check(lib().lagp_predict_mle(design, _ptr(XX), XX.shape[0], _ptr(cand_idx), ctypes.byref(params),
                                         ctypes.byref(mle), _ptr(mean), _ptr(s2), _ptr(df), _ptr(dhat),
                                         _ptr(sel_idx), _ptr(iters), _ptr(status), _stream(stream)))


def lagp_fit_separable(XS, yS, g: float, theta0, dmin: float, dmax: float, tol: float = 0.0, maxit: int = 0,
                       maxsweep: int = 0, stream=None):
    """Global separable lengthscales on the subset (XS, yS) (device tensors):
    returns (theta numpy (p,), evaluations, status bits)."""
    n, p = XS.shape
    th = np.ascontiguousarray(np.broadcast_to(np.atleast_1d(np.asarray(theta0, dtype=np.float64)), (p,))).copy()
    it, st = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().lagp_fit_separable(_ptr(XS), _ptr(yS), n, p, g, th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    dmin, dmax, tol, maxit, maxsweep, ctypes.byref(it), ctypes.byref(st),
                                    _stream(stream)))
    return th, it.value, st.value


def lagp_prescale(X, theta, out, stream=None) -> int:
    """out = X / sqrt(theta) per column (device tensors, N x p)."""
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    return _check(lib().lagp_prescale(_ptr(X), X.shape[0], X.shape[1],
                                      th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(out), _stream(stream)))


def lagp_server_create(design, hbm_budget_bytes: int, max_inflight: int):
    h = _vp()
    _check(lib().lagp_server_create(design, int(hbm_budget_bytes), int(max_inflight), ctypes.byref(h)))
    return h


def lagp_server_submit(server, XX_host: np.ndarray, params: lagp_params) -> tuple[int, int]:
    XX_host = np.ascontiguousarray(XX_host, dtype=np.float64)
    t = ctypes.c_uint64()
    rc = lib().lagp_server_submit(server, XX_host.ctypes.data, XX_host.shape[0], ctypes.byref(params), ctypes.byref(t))
    if rc == LAGP_EAGAIN:
        return rc, 0
    _check(rc)
    return rc, t.value


def lagp_server_poll(server, ticket: int) -> bool:
    done = ctypes.c_int32()
    _check(lib().lagp_server_poll(server, ctypes.c_uint64(ticket), ctypes.byref(done)))
    return bool(done.value)


def lagp_server_fetch(server, ticket: int, M: int, n: int):
    out = dict(mean=np.empty(M), s2=np.empty(M), df=np.empty(M), sel=np.empty((M, n), np.int32),
               status=np.empty(M, np.int32))
    lat = ctypes.c_double()
    rc = lib().lagp_server_fetch(server, ctypes.c_uint64(ticket), out["mean"].ctypes.data, out["s2"].ctypes.data,
                                 out["df"].ctypes.data, out["sel"].ctypes.data, out["status"].ctypes.data,
                                 ctypes.byref(lat))
    _check(rc)
    out["latency_ms"] = lat.value
    out["rc"] = rc
    return out


def lagp_server_stats(server, reset: bool = False):
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().lagp_server_stats(server, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), int(reset)))
    return dict(p50_ms=a.value, p99_ms=b.value, pred_per_s=c.value)


def lagp_server_destroy(server) -> None:
    lib().lagp_server_destroy(server)


# ------------------------------------------------------------ convenience --

def _torch_stream(stream):
    """The torch stream object for a stream argument (None: the current one)."""
    import torch

    if stream is None:
        return torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return stream
    return torch.cuda.ExternalStream(int(getattr(stream, "cuda_stream", stream)))


def _on_stream(stream, *tensors):
    """Order work on `stream` after torch's current stream (which produced
    the converted inputs) and tell the caching allocator that the tensors are
    in use on `stream`, so that none of them is reused while the library's
    kernels still read or write it."""
    import torch

    s = _torch_stream(stream)
    cur = torch.cuda.current_stream()
    if s.cuda_stream != cur.cuda_stream:
        s.wait_stream(cur)
        for t in tensors:
            if t is not None:
                t.record_stream(s)
    return s

class Design:
    """Owns a lagp_design handle for torch tensors X (N x p), y (N)."""

    def __init__(self, X, y, stream=None):
        import torch

        self.X = torch.as_tensor(X, dtype=torch.float64, device="cuda").contiguous()
        self.y = torch.as_tensor(y, dtype=torch.float64, device="cuda").contiguous()
        self.handle = lagp_design_create(self.X, self.y, _on_stream(stream, self.X, self.y))
        self.N, self.p = self.X.shape

    def close(self):
        if self.handle is not None:
            lagp_design_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def candidates(self, XX, ncand: int, stream=None):
        import torch

        XX = torch.as_tensor(XX, dtype=torch.float64, device="cuda").contiguous()
        idx = torch.empty((XX.shape[0], ncand), dtype=torch.int32, device="cuda")
        d2 = torch.empty((XX.shape[0], ncand), dtype=torch.float64, device="cuda")
        s = _on_stream(stream, XX, idx, d2)
        lagp_candidates(self.handle, XX, ncand, idx, d2, s)
        return idx, d2

    def predict(self, XX, params, stream=None, sel=True, diag=True, counts=False):
        """Returns a dict of device tensors: mean, s2, df, sel, diag, status
        (and counts, the per-step search work, when asked for)."""
        import torch

        XX = torch.as_tensor(XX, dtype=torch.float64, device="cuda").contiguous()
        P = params if isinstance(params, lagp_params) else make_params(params)
        M = XX.shape[0]
        n0 = P.n if P.search == LAGP_SEARCH_NN else P.n0
        dev = dict(dtype=torch.float64, device="cuda")
        out = dict(mean=torch.empty(M, **dev), s2=torch.empty(M, **dev), df=torch.empty(M, **dev),
                   status=torch.empty(M, dtype=torch.int32, device="cuda"))
        out["sel"] = torch.empty((M, P.n), dtype=torch.int32, device="cuda") if sel else None
        out["diag"] = torch.empty((M, P.n - n0, 2), **dev) if diag else None
        if counts:
            out["counts"] = torch.empty((M, P.n - n0, 2), dtype=torch.int32, device="cuda")
        s = _on_stream(stream, XX, *out.values())
        if counts:
            lagp_predict_counts(self.handle, XX, None, P, out["mean"], out["s2"], out["df"], out["sel"], out["diag"],
                                out["status"], out["counts"], s)
        else:
            lagp_predict(self.handle, XX, P, out["mean"], out["s2"], out["df"], out["sel"], out["diag"],
                         out["status"], s)
        return out

    def predict_mle(self, XX, params, mode: int, dmin: float = 0.0, dmax: float = 0.0, tol: float = 0.0,
                    maxit: int = 0, stream=None):
        """Local MLE prediction: a dict of device tensors mean, s2, df, dhat,
        sel, iters, status."""
        import torch

        XX = torch.as_tensor(XX, dtype=torch.float64, device="cuda").contiguous()
        P = params if isinstance(params, lagp_params) else make_params(params)
        Q = make_mle_params(mode, dmin, dmax, tol, maxit)
        M = XX.shape[0]
        dev = dict(dtype=torch.float64, device="cuda")
        i32 = dict(dtype=torch.int32, device="cuda")
        out = dict(mean=torch.empty(M, **dev), s2=torch.empty(M, **dev), df=torch.empty(M, **dev),
                   dhat=torch.empty(M, **dev), sel=torch.empty((M, P.n), **i32), iters=torch.empty(M, **i32),
                   status=torch.empty(M, **i32))
        s = _on_stream(stream, XX, *out.values())
        lagp_predict_mle(self.handle, XX, None, P, Q, out["mean"], out["s2"], out["df"], out["dhat"], out["sel"],
                         out["iters"], out["status"], s)
        return out
