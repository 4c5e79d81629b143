"""ORACLE -- test infrastructure only.

Python access (ctypes) to the plain FP64 single-threaded C oracle in
``oracle.c``: normalised PDFs, the NLL of Eq. 1 with its analytic gradient
and Hessian, and a BFGS fit with the inverse-Hessian covariance.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It never imports the GPU package, and
the GPU package never imports it.

Model descriptions are plain dicts (the same plain data the GPU binding
accepts, converted here into the oracle's own C structs)::

    {"dims":   [{"name": "m", "lo": 5.0, "hi": 5.6}, ...],
     "params": [{"name": "mu", "value": 5.28, "fixed": False}, ...],
     "nodes":  [{"kind": "gauss", "dims": [0], "params": [0, 1]},
                {"kind": "exp",   "dims": [0], "params": [2]},
                {"kind": "sum",   "children": [0, 1], "params": [3]}],
     "root": 2}
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_KINDS = {"gauss": 1, "exp": 2, "cheb": 3, "pwave": 4, "prod": 5, "sum": 6}
MAXP = 32


class _Node(C.Structure):
    _fields_ = [("kind", C.c_int), ("dim", C.c_int * 3), ("npar", C.c_int),
                ("par", C.c_int * 8), ("nchild", C.c_int), ("child", C.c_int * 4)]


class _Model(C.Structure):
    _fields_ = [("ndim", C.c_int), ("lo", C.c_double * 8), ("hi", C.c_double * 8),
                ("nnode", C.c_int), ("node", _Node * 64), ("root", C.c_int),
                ("npar", C.c_int)]


class _FitOpts(C.Structure):
    _fields_ = [("edm_tol", C.c_double), ("max_iter", C.c_int), ("polish", C.c_int)]


class _FitInfo(C.Structure):
    _fields_ = [("nll", C.c_double), ("edm", C.c_double), ("n_iter", C.c_int),
                ("n_eval", C.c_int), ("status", C.c_int)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = C.CDLL(_build.LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        lib.orc_model_init.argtypes = [C.POINTER(_Model), C.c_int, dp, dp, C.c_int, ip,
                                       C.c_int, C.c_int]
        lib.orc_model_init.restype = C.c_int
        lib.orc_pdf.argtypes = [C.POINTER(_Model), C.c_long, dp, dp, dp]
        lib.orc_pdf.restype = None
        lib.orc_nll.argtypes = [C.POINTER(_Model), C.c_long, dp, dp, dp, C.c_int, dp, dp, dp]
        lib.orc_nll.restype = C.c_long
        lib.orc_w2.argtypes = [C.POINTER(_Model), C.c_long, dp, dp, dp, dp]
        lib.orc_w2.restype = C.c_long
        u64p = C.POINTER(C.c_uint64)
        lib.orc_philox4x64.argtypes = [u64p, u64p, u64p]
        lib.orc_philox4x64.restype = None
        lib.orc_generate.argtypes = [C.POINTER(_Model), C.c_long, C.c_long, C.c_uint64, dp, dp]
        lib.orc_generate.restype = C.c_long
        lib.orc_fit.argtypes = [C.POINTER(_Model), C.c_long, dp, dp, dp, ip,
                                C.POINTER(_FitOpts), dp, C.POINTER(_FitInfo)]
        lib.orc_fit.restype = C.c_int
        _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def philox4x64(ctr, key):
    """One Philox4x64-10 block: four 64-bit words from a counter (4 words)
    and a key (2 words)."""
    c = (C.c_uint64 * 4)(*[int(v) for v in ctr])
    k = (C.c_uint64 * 2)(*[int(v) for v in key])
    o = (C.c_uint64 * 4)()
    _load().orc_philox4x64(c, k, o)
    return [int(v) for v in o]


def _ncols(x, ndim):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if x.ndim == 1:
        x = x.reshape(1, -1)
    if x.shape[0] != ndim:
        raise ValueError(f"events must be shaped (ndim={ndim}, n), got {x.shape}")
    return x


class Model:
    """The oracle's view of a model description (see module docstring)."""

    def __init__(self, desc):
        lib = _load()
        self.desc = desc
        self.ndim = len(desc["dims"])
        self.npar = len(desc["params"])
        lo = np.array([d["lo"] for d in desc["dims"]], dtype=np.float64)
        hi = np.array([d["hi"] for d in desc["dims"]], dtype=np.float64)
        rows = []
        for nd in desc["nodes"]:
            r = [0] * 18
            r[0] = _KINDS[nd["kind"]]
            for k, d in enumerate(nd.get("dims", [])):
                r[1 + k] = d
            ps = nd.get("params", [])
            r[4] = len(ps)
            for k, p in enumerate(ps):
                r[5 + k] = p
            ch = nd.get("children", [])
            r[13] = len(ch)
            for k, c in enumerate(ch):
                r[14 + k] = c
            rows += r
        nodes = np.array(rows, dtype=np.int32)
        self._m = _Model()
        rc = lib.orc_model_init(C.byref(self._m), self.ndim, _dptr(lo), _dptr(hi),
                                len(desc["nodes"]),
                                nodes.ctypes.data_as(C.POINTER(C.c_int)),
                                int(desc["root"]), self.npar)
        if rc != 0:
            raise ValueError(f"oracle rejected the model description (code {rc})")
        self.theta0 = np.array([p["value"] for p in desc["params"]], dtype=np.float64)
        self.free = np.array([not p.get("fixed", False) for p in desc["params"]])

    def pdf(self, x, theta=None):
        x = _ncols(x, self.ndim)
        th = np.ascontiguousarray(self.theta0 if theta is None else theta, dtype=np.float64)
        out = np.empty(x.shape[1], dtype=np.float64)
        _load().orc_pdf(C.byref(self._m), x.shape[1], _dptr(x), _dptr(th), _dptr(out))
        return out

    def nll(self, x, theta=None, w=None, order=0):
        """Returns (nll, grad[npar] or None, hess[npar, npar] or None, n_bad)."""
        x = _ncols(x, self.ndim)
        n = x.shape[1]
        th = np.ascontiguousarray(self.theta0 if theta is None else theta, dtype=np.float64)
        wp = None
        if w is not None:
            w = np.ascontiguousarray(w, dtype=np.float64)
            if w.shape != (n,):
                raise ValueError("weights must have one entry per event")
            wp = _dptr(w)
        nll = C.c_double()
        g = np.zeros(self.npar)
        h = np.zeros((self.npar, self.npar))
        bad = _load().orc_nll(C.byref(self._m), n, _dptr(x), wp, _dptr(th), order,
                              C.byref(nll), _dptr(g), _dptr(h))
        return (nll.value, g if order >= 1 else None, h if order >= 2 else None, int(bad))

    def w2(self, x, theta=None, w=None):
        """W2 = sum_i w_i^2 s_i s_i^T over all parameters; returns (w2, n_bad)."""
        x = _ncols(x, self.ndim)
        n = x.shape[1]
        th = np.ascontiguousarray(self.theta0 if theta is None else theta, dtype=np.float64)
        wp = None
        if w is not None:
            w = np.ascontiguousarray(w, dtype=np.float64)
            if w.shape != (n,):
                raise ValueError("weights must have one entry per event")
            wp = _dptr(w)
        out = np.zeros((self.npar, self.npar))
        bad = _load().orc_w2(C.byref(self._m), n, _dptr(x), wp, _dptr(th), _dptr(out))
        return out, int(bad)

    def generate(self, n, seed, theta=None, i0=0):
        """Events i0 .. i0+n-1 of pseudo-experiment `seed` at theta: (ndim, n)
        FP64 and the number of events that hit the attempt cap."""
        th = np.ascontiguousarray(self.theta0 if theta is None else theta, dtype=np.float64)
        out = np.zeros((self.ndim, n))
        bad = _load().orc_generate(C.byref(self._m), int(i0), int(n), C.c_uint64(seed), _dptr(th),
                                   _dptr(out))
        return out, int(bad)

    def fit(self, x, start=None, free=None, w=None, edm_tol=1e-6, max_iter=500, polish=0):
        """BFGS fit; returns a dict with theta, errors, cov (free order), nll, edm ..."""
        x = _ncols(x, self.ndim)
        n = x.shape[1]
        th = np.array(self.theta0 if start is None else start, dtype=np.float64)
        fm = np.ascontiguousarray(self.free if free is None else free, dtype=np.int32)
        nf = int(fm.sum())
        cov = np.zeros((nf, nf))
        wp = None
        if w is not None:
            w = np.ascontiguousarray(w, dtype=np.float64)
            wp = _dptr(w)
        opts = _FitOpts(edm_tol, max_iter, polish)
        info = _FitInfo()
        _load().orc_fit(C.byref(self._m), n, _dptr(x), wp, _dptr(th),
                        fm.ctypes.data_as(C.POINTER(C.c_int)), C.byref(opts), _dptr(cov),
                        C.byref(info))
        err = np.sqrt(np.maximum(np.diag(cov), 0.0))
        return {"theta": th, "errors": err, "cov": cov, "nll": info.nll, "edm": info.edm,
                "n_iter": info.n_iter, "n_eval": info.n_eval, "status": info.status,
                "free": fm.astype(bool)}
