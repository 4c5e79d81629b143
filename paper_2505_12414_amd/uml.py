"""Python binding of libuml (ctypes; argument marshalling only).

Every function here calls the C ABI declared in include/uml.h under the same
name; all arithmetic runs in the library's HIP kernels.  The library must
have been built (``python -m paper_2505_12414_amd.build``); loading fails
loudly otherwise -- there is no CPU fallback.

Model descriptions are plain dicts::

    {"dims":   [{"name": "m", "lo": 5.0, "hi": 5.6}, ...],
     "params": [{"name": "mu", "value": 5.28, "fixed": False}, ...],
     "nodes":  [{"kind": "gauss", "dims": [0], "params": [0, 1]}, ...,
                {"kind": "sum", "children": [0, 1], "params": [3]}],
     "root": 2}
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libuml.so")

UML_OK = 0
UML_E_INVALID = -1
UML_E_UNSUPPORTED = -2
UML_E_EVENT_DOMAIN = -3
UML_E_PDF_NONPOSITIVE = -4
UML_E_HIP = -5
UML_E_NOMEM = -6
UML_E_NOT_PD = -7
UML_E_BUDGET = -8
UML_E_QUEUE_FULL = -9
UML_E_TIMEOUT = -10
UML_E_GENERATION = -11

UML_FP64, UML_MIXED = 0, 1
UML_F32, UML_F64 = 0, 1
UML_DATA_DEVICE_SRC = 1
UML_DATA_BORROW = 2
MAX_PARAMS = 32

KINDS = {"gauss": 1, "exp": 2, "cheb": 3, "pwave": 4, "prod": 5, "sum": 6}
FIT_STATUS = {0: "converged", 1: "max_iter", 2: "linesearch_fail", 3: "hessian_not_pd",
              4: "pdf_nonpositive", 5: "cancelled", 6: "generation_failed"}


class UmlError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class uml_dim(C.Structure):
    _fields_ = [("lo", C.c_double), ("hi", C.c_double)]


class uml_param(C.Structure):
    _fields_ = [("value", C.c_double), ("lo", C.c_double), ("hi", C.c_double),
                ("fixed", C.c_int32)]


class uml_node(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dims", C.c_int32 * 3), ("n_params", C.c_int32),
                ("params", C.c_int32 * 8), ("n_children", C.c_int32),
                ("children", C.c_int32 * 4)]


UML_MODEL_PRECOMPUTE_ANGULAR = 1


class uml_model_desc(C.Structure):
    _fields_ = [("n_dims", C.c_int32), ("dims", C.POINTER(uml_dim)),
                ("n_params", C.c_int32), ("params", C.POINTER(uml_param)),
                ("n_nodes", C.c_int32), ("nodes", C.POINTER(uml_node)),
                ("root", C.c_int32), ("precision", C.c_int32), ("flags", C.c_int32)]


class uml_fit_options(C.Structure):
    _fields_ = [("edm_tol", C.c_double), ("max_iter", C.c_int32), ("polish", C.c_int32),
                ("want_cov", C.c_int32), ("cov_kind", C.c_int32), ("method", C.c_int32)]


class uml_fit_result(C.Structure):
    _fields_ = [("params", C.c_double * MAX_PARAMS), ("errors", C.c_double * MAX_PARAMS),
                ("cov", C.c_double * (MAX_PARAMS * MAX_PARAMS)), ("nll", C.c_double),
                ("edm", C.c_double), ("n_free", C.c_int32), ("n_iter", C.c_int32),
                ("n_eval", C.c_int32), ("status", C.c_int32), ("ticket", C.c_uint64),
                ("latency_s", C.c_double), ("n_bad_events", C.c_int64)]


class uml_server_options(C.Structure):
    _fields_ = [("max_slots", C.c_int32), ("hbm_budget", C.c_int64),
                ("max_pending", C.c_int32), ("fit", uml_fit_options)]


class uml_request(C.Structure):
    _fields_ = [("n_events", C.c_int64), ("cols", C.POINTER(C.c_void_p)), ("dtype", C.c_int32),
                ("w", C.c_void_p), ("start", C.POINTER(C.c_double)), ("generate", C.c_int32),
                ("seed", C.c_uint64), ("gen_theta", C.POINTER(C.c_double))]


class uml_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("finished", C.c_int64),
                ("pending", C.c_int64), ("active", C.c_int64), ("iterations", C.c_int64),
                ("resident_bytes", C.c_int64), ("peak_resident_bytes", C.c_int64),
                ("budget_waits", C.c_int64), ("t_admit_s", C.c_double), ("t_iterate_s", C.c_double),
                ("t_retire_s", C.c_double)]


# name -> (restype, argtypes)
_P = C.c_void_p
_DP = C.POINTER(C.c_double)
SIGNATURES = {
    "uml_model_create": (C.c_int, [C.POINTER(uml_model_desc), C.POINTER(_P)]),
    "uml_model_destroy": (None, [_P]),
    "uml_model_n_free": (C.c_int, [_P]),
    "uml_model_describe": (C.c_int, [_P, C.c_char_p, C.c_int32]),
    "uml_data_create": (C.c_int, [_P, C.c_int64, C.POINTER(C.c_void_p), C.c_int32, _P,
                                  C.c_int32, _P, C.POINTER(_P)]),
    "uml_data_destroy": (None, [_P]),
    "uml_data_generate": (C.c_int, [_P, C.c_int64, C.c_uint64, _DP, _P, C.POINTER(_P)]),
    "uml_data_download": (C.c_int, [_P, C.POINTER(C.c_void_p), _P]),
    "uml_data_n_events": (C.c_int64, [_P]),
    "uml_eval_nll": (C.c_int, [_P, _P, _DP, _DP, _P]),
    "uml_eval_nll_grad": (C.c_int, [_P, _P, _DP, _DP, _DP, _P]),
    "uml_eval_nll_grad_dev": (C.c_int, [_P, _P, _P, _P, _P]),
    "uml_eval_nll_grad_noalloc": (C.c_int, [_P, C.c_int64, C.POINTER(_P), _P, _P, _P, _P]),
    "uml_eval_hessian": (C.c_int, [_P, _P, _DP, _DP, _DP, _DP, _DP, _P]),
    "uml_eval_bad_events": (C.c_int, [_P, _P, _DP, C.POINTER(C.c_int64), _P]),
    "uml_fit_options_default": (None, [C.POINTER(uml_fit_options)]),
    "uml_fit": (C.c_int, [_P, _P, _DP, C.POINTER(uml_fit_options), C.POINTER(uml_fit_result)]),
    "uml_fit_batch": (C.c_int, [_P, C.POINTER(_P), C.c_int32, _DP, C.POINTER(uml_fit_options),
                                C.POINTER(uml_fit_result)]),
    "uml_server_options_default": (None, [C.POINTER(uml_server_options)]),
    "uml_server_create": (C.c_int, [_P, C.POINTER(uml_server_options), C.POINTER(_P)]),
    "uml_server_submit": (C.c_int, [_P, C.POINTER(uml_request), C.POINTER(C.c_uint64)]),
    "uml_server_poll": (C.c_int, [_P, C.POINTER(uml_fit_result), C.c_int32,
                                  C.POINTER(C.c_int32), C.c_int32]),
    "uml_server_stats_get": (C.c_int, [_P, C.POINTER(uml_server_stats)]),
    "uml_server_drain": (C.c_int, [_P]),
    "uml_server_destroy": (None, [_P]),
    "uml_last_error": (C.c_char_p, []),
    "uml_version": (C.c_char_p, []),
}

_lib = None


def _preload_torch_hip_runtime():
    """Loads the HIP runtime bundled with PyTorch before libuml, so that
    libuml, torch's streams and torch's device memory share one runtime
    (both runtimes carry the soname libamdhip64.so.7; the first one loaded
    serves every later user in the process)."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.origin:
        return None
    path = os.path.join(os.path.dirname(spec.origin), "lib", "libamdhip64.so")
    if os.path.exists(path):
        return C.CDLL(path, mode=C.RTLD_GLOBAL)
    return None


def lib():
    """The loaded libuml.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2505_12414_amd.build` (no CPU fallback exists)")
        _preload_torch_hip_runtime()
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error():
    return lib().uml_last_error().decode()


def check(rc, allow=()):
    if rc != UML_OK and rc not in allow:
        raise UmlError(rc, last_error())
    return rc


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


def _dptr(a):
    return a.ctypes.data_as(_DP)


class Model:
    """uml_model_create / uml_model_destroy."""

    def __init__(self, desc, precision="mixed", precompute=False):
        """precompute: store the P-wave's event-only terms as extra columns
        (UML_MODEL_PRECOMPUTE_ANGULAR) instead of recomputing them."""
        self.desc = desc
        self.precompute = bool(precompute)
        prec = {"mixed": UML_MIXED, "fp64": UML_FP64}[precision]
        self.precision = precision
        dims = (uml_dim * len(desc["dims"]))(*[uml_dim(d["lo"], d["hi"]) for d in desc["dims"]])
        ps = desc["params"]
        params = (uml_param * max(1, len(ps)))(*[
            uml_param(p["value"], p.get("lo", -1e30), p.get("hi", 1e30), int(p.get("fixed", False)))
            for p in ps])
        nodes = (uml_node * len(desc["nodes"]))()
        for i, nd in enumerate(desc["nodes"]):
            n = nodes[i]
            n.kind = KINDS[nd["kind"]]
            for k, d in enumerate(nd.get("dims", [])):
                n.dims[k] = d
            pp = nd.get("params", [])
            n.n_params = len(pp)
            for k, p in enumerate(pp):
                n.params[k] = p
            ch = nd.get("children", [])
            n.n_children = len(ch)
            for k, c in enumerate(ch):
                n.children[k] = c
        d = uml_model_desc(len(desc["dims"]), dims, len(ps), params, len(desc["nodes"]), nodes,
                           int(desc["root"]), prec, UML_MODEL_PRECOMPUTE_ANGULAR if precompute else 0)
        h = _P()
        check(lib().uml_model_create(C.byref(d), C.byref(h)))
        self.handle = h
        self.n_params = len(ps)
        self.n_dims = len(desc["dims"])
        self.n_free = lib().uml_model_n_free(h)
        self.free = np.array([not p.get("fixed", False) for p in ps])
        self.theta0 = np.array([p["value"] for p in ps], dtype=np.float64)

    def describe(self):
        buf = C.create_string_buffer(4096)
        check(lib().uml_model_describe(self.handle, buf, 4096))
        return buf.value.decode()

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.uml_model_destroy(self.handle)
            self.handle = None


class Data:
    """uml_data_create / uml_data_destroy.  events: array (n_dims, n) of
    float32 or float64 (host numpy, or a torch CUDA tensor for device upload).
    borrow=True (CUDA tensors only, UML_DATA_BORROW): the dataset reads the
    tensor's rows in place; they must have the model's storage type and start
    on 16-byte boundaries (n a multiple of 4 for FP32 rows, of 2 for FP64), and
    this object keeps the tensors alive."""

    def __init__(self, model, events, weights=None, stream=None, borrow=False):
        self.model = model
        flags = 0
        keep = []
        self._keep = None
        if hasattr(events, "is_cuda") and events.is_cuda:
            import torch
            ev = events.contiguous()
            if ev.dim() == 1:
                ev = ev.reshape(1, -1)
            dtype = UML_F32 if ev.dtype == torch.float32 else UML_F64
            if ev.dtype not in (torch.float32, torch.float64):
                raise TypeError("events must be float32 or float64")
            n = ev.shape[1]
            cols = (C.c_void_p * ev.shape[0])(*[ev[d].data_ptr() for d in range(ev.shape[0])])
            wptr = None
            if weights is not None:
                wt = weights.to(ev.dtype).contiguous()
                keep.append(wt)
                wptr = wt.data_ptr()
            flags |= UML_DATA_DEVICE_SRC
            keep.append(ev)
            if borrow:
                flags |= UML_DATA_BORROW
                self._keep = keep
        else:
            if borrow:
                raise ValueError("borrow=True needs CUDA tensors")
            ev = np.asarray(events)
            if ev.ndim == 1:
                ev = ev.reshape(1, -1)
            if ev.dtype not in (np.float32, np.float64):
                ev = ev.astype(np.float64)
            if ev.shape[1] > 1 and ev.strides[1] != ev.itemsize:
                ev = np.ascontiguousarray(ev)
            dtype = UML_F32 if ev.dtype == np.float32 else UML_F64
            n = ev.shape[1]
            cols = (C.c_void_p * ev.shape[0])(*[ev[d].ctypes.data for d in range(ev.shape[0])])
            wptr = None
            if weights is not None:
                wt = np.ascontiguousarray(np.asarray(weights, dtype=ev.dtype))
                if wt.shape != (n,):
                    raise ValueError("weights must have one entry per event")
                keep.append(wt)
                wptr = wt.ctypes.data
            keep.append(ev)
        if ev.shape[0] != model.n_dims:
            raise ValueError(f"events must have {model.n_dims} rows")
        h = _P()
        check(lib().uml_data_create(model.handle, n, cols, dtype, wptr, flags, _stream_ptr(stream),
                                    C.byref(h)))
        self.handle = h
        self.n = n
        self.weighted = weights is not None

    @classmethod
    def generate(cls, model, n, seed, theta=None, stream=None):
        """uml_data_generate: a pseudo-experiment of n events drawn on the device
        from the model at theta (default: the description's values)."""
        obj = cls.__new__(cls)
        obj.model = model
        th = None if theta is None else np.ascontiguousarray(theta, dtype=np.float64)
        h = _P()
        check(lib().uml_data_generate(model.handle, int(n), C.c_uint64(int(seed)),
                                      None if th is None else _dptr(th), _stream_ptr(stream),
                                      C.byref(h)))
        obj.handle = h
        obj.n = int(n)
        obj.weighted = False
        return obj

    def download(self):
        """The stored event columns, (n_dims, n), FP32 for mixed models."""
        dt = np.float32 if self.model.precision == "mixed" else np.float64
        out = np.zeros((self.model.n_dims, self.n), dtype=dt)
        cols = (C.c_void_p * self.model.n_dims)(*[out[d].ctypes.data for d in range(self.model.n_dims)])
        check(lib().uml_data_download(self.handle, cols, None))
        return out

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.uml_data_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


def _theta(model, theta):
    th = np.ascontiguousarray(model.theta0 if theta is None else theta, dtype=np.float64)
    if th.shape != (model.n_params,):
        raise ValueError(f"theta must hold all {model.n_params} parameters")
    return th


def uml_eval_nll(model, data, theta=None, stream=None, allow_nonpositive=True):
    th = _theta(model, theta)
    out = C.c_double()
    check(lib().uml_eval_nll(model.handle, data.handle, _dptr(th), C.byref(out),
                             _stream_ptr(stream)),
          allow=(UML_E_PDF_NONPOSITIVE,) if allow_nonpositive else ())
    return out.value


def uml_eval_nll_grad(model, data, theta=None, stream=None, allow_nonpositive=True):
    """Returns (nll, gradient over the free parameters)."""
    th = _theta(model, theta)
    out = C.c_double()
    g = np.zeros(max(1, model.n_free))
    check(lib().uml_eval_nll_grad(model.handle, data.handle, _dptr(th), C.byref(out), _dptr(g),
                                  _stream_ptr(stream)),
          allow=(UML_E_PDF_NONPOSITIVE,) if allow_nonpositive else ())
    return out.value, g[:model.n_free].copy()


def uml_eval_bad_events(model, data, theta=None, stream=None):
    """Events at which P <= 0 or P is not finite (all of them outside the
    model's domain)."""
    th = _theta(model, theta)
    out = C.c_int64()
    check(lib().uml_eval_bad_events(model.handle, data.handle, _dptr(th), C.byref(out),
                                    _stream_ptr(stream)))
    return int(out.value)


def uml_eval_nll_grad_dev(model, data, d_theta, d_out, stream=None):
    """Stream-ordered: d_theta (float64 CUDA tensor, n_params) -> d_out
    (float64 CUDA tensor, 1 + n_free).  stream: torch.cuda.Stream, raw
    hipStream_t int, or None for torch's current stream."""
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    check(lib().uml_eval_nll_grad_dev(model.handle, data.handle, d_theta.data_ptr(),
                                      d_out.data_ptr(), _stream_ptr(stream)))


def uml_eval_nll_grad_noalloc(model, n, d_cols, d_w, d_theta, d_out, stream=None):
    """Stream-ordered, allocation-free: n events in the device columns d_cols
    (sequence of n_dims CUDA tensors, or raw device addresses), optional
    weights d_w, d_theta -> d_out as uml_eval_nll_grad_dev."""
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()

    def addr(t):
        return t if isinstance(t, int) else t.data_ptr()
    cols = (_P * len(d_cols))(*[addr(c) for c in d_cols])
    check(lib().uml_eval_nll_grad_noalloc(model.handle, int(n), cols,
                                          None if d_w is None else addr(d_w), addr(d_theta),
                                          addr(d_out), _stream_ptr(stream)))


def uml_eval_hessian(model, data, theta=None, want_w2=False, stream=None, allow_nonpositive=True):
    """Returns (nll, grad, hess[, w2]) over the free parameters."""
    th = _theta(model, theta)
    nf = model.n_free
    out = C.c_double()
    g = np.zeros(max(1, nf))
    h = np.zeros(max(1, nf * nf))
    w2 = np.zeros(max(1, nf * nf)) if want_w2 else None
    check(lib().uml_eval_hessian(model.handle, data.handle, _dptr(th), C.byref(out), _dptr(g),
                                 _dptr(h), _dptr(w2) if want_w2 else None, _stream_ptr(stream)),
          allow=(UML_E_PDF_NONPOSITIVE,) if allow_nonpositive else ())
    res = (out.value, g[:nf].copy(), h[:nf * nf].reshape(nf, nf).copy())
    return res + ((w2[:nf * nf].reshape(nf, nf).copy(),) if want_w2 else ())


UML_COV_HESSE, UML_COV_SANDWICH = 0, 1
UML_METHOD_BFGS, UML_METHOD_NEWTON = 0, 1


def fit_options(edm_tol=1e-6, max_iter=1000, polish=0, want_cov=1, cov_kind=UML_COV_HESSE,
                method=UML_METHOD_BFGS):
    o = uml_fit_options()
    lib().uml_fit_options_default(C.byref(o))
    o.edm_tol, o.max_iter, o.polish, o.want_cov = edm_tol, max_iter, polish, want_cov
    o.cov_kind, o.method = cov_kind, method
    return o


def result_dict(model, r):
    nf = r.n_free
    return {"theta": np.array(r.params[:model.n_params]),
            "errors": np.array(r.errors[:model.n_params]),
            "cov": np.array(r.cov[:nf * nf]).reshape(nf, nf), "nll": r.nll, "edm": r.edm,
            "n_iter": r.n_iter, "n_eval": r.n_eval, "status": r.status,
            "status_name": FIT_STATUS.get(r.status, str(r.status)), "ticket": r.ticket,
            "latency_s": r.latency_s, "n_bad_events": r.n_bad_events}


def uml_fit(model, data, start=None, **opts):
    th = _theta(model, start)
    o = fit_options(**opts)
    r = uml_fit_result()
    check(lib().uml_fit(model.handle, data.handle, _dptr(th), C.byref(o), C.byref(r)))
    return result_dict(model, r)


def uml_fit_batch(model, datas, starts=None, **opts):
    n = len(datas)
    st = np.ascontiguousarray(np.tile(model.theta0, (n, 1)) if starts is None else starts,
                              dtype=np.float64)
    hs = (_P * n)(*[d.handle for d in datas])
    o = fit_options(**opts)
    rs = (uml_fit_result * n)()
    check(lib().uml_fit_batch(model.handle, hs, n, _dptr(st), C.byref(o), rs))
    return [result_dict(model, r) for r in rs]


def uml_version():
    return lib().uml_version().decode()


class Server:
    """uml_server_*: a device-resident loop fitting many pseudo-experiments of
    one model with continuous batching."""

    def __init__(self, model, max_slots=256, hbm_budget=4 << 30, max_pending=1 << 20, **fit_opts):
        o = uml_server_options()
        lib().uml_server_options_default(C.byref(o))
        o.max_slots, o.hbm_budget, o.max_pending = max_slots, hbm_budget, max_pending
        o.fit = fit_options(**fit_opts)
        h = _P()
        check(lib().uml_server_create(model.handle, C.byref(o), C.byref(h)))
        self.handle = h
        self.model = model
        self._buf = (uml_fit_result * 256)()   # reused by poll

    def submit(self, events, weights=None, start=None):
        """events: (n_dims, n) float32/float64 host array.  Returns the ticket."""
        ev = np.asarray(events)
        if ev.ndim == 1:
            ev = ev.reshape(1, -1)
        if ev.dtype not in (np.float32, np.float64):
            ev = ev.astype(np.float64)
        if ev.shape[1] > 1 and ev.strides[1] != ev.itemsize:
            ev = np.ascontiguousarray(ev)   # rows must be contiguous; views of rows are not copied
        cols = (C.c_void_p * ev.shape[0])(*[ev[d].ctypes.data for d in range(ev.shape[0])])
        wt = None
        if weights is not None:
            wt = np.ascontiguousarray(np.asarray(weights, dtype=ev.dtype))
        st = None if start is None else np.ascontiguousarray(start, dtype=np.float64)
        q = uml_request(ev.shape[1], cols, UML_F32 if ev.dtype == np.float32 else UML_F64,
                        None if wt is None else wt.ctypes.data, None if st is None else _dptr(st))
        t = C.c_uint64()
        check(lib().uml_server_submit(self.handle, C.byref(q), C.byref(t)))
        return t.value

    def submit_generated(self, n, seed, gen_theta=None, start=None):
        """A pseudo-experiment of n events drawn on the device (seed, at
        gen_theta or the model's values) and fitted from start."""
        st = None if start is None else np.ascontiguousarray(start, dtype=np.float64)
        gt = None if gen_theta is None else np.ascontiguousarray(gen_theta, dtype=np.float64)
        q = uml_request(int(n), None, UML_F64, None, None if st is None else _dptr(st), 1,
                        C.c_uint64(int(seed)), None if gt is None else _dptr(gt))
        t = C.c_uint64()
        check(lib().uml_server_submit(self.handle, C.byref(q), C.byref(t)))
        return t.value

    def poll(self, max_results=256, timeout_us=0):
        """Up to max_results finished fits (at most 256 per call)."""
        rs = self._buf
        k = max(1, min(int(max_results), len(rs)))
        n = C.c_int32()
        rc = lib().uml_server_poll(self.handle, rs, k, C.byref(n), timeout_us)
        check(rc, allow=(UML_E_TIMEOUT,))
        return [result_dict(self.model, rs[i]) for i in range(n.value)]

    def drain(self):
        check(lib().uml_server_drain(self.handle))

    def stats(self):
        st = uml_server_stats()
        check(lib().uml_server_stats_get(self.handle, C.byref(st)))
        return {k: getattr(st, k) for k, _ in uml_server_stats._fields_}

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.uml_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()
