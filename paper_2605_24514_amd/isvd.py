"""Python binding of libisvd.so (ctypes): argument marshalling only.

Every step of an update, refresh or tick runs in the library's HIP kernels;
this module converts numpy arrays / torch tensors into pointers and checks
status codes.  It fails loudly if the library is missing: there is no
fallback implementation.
"""
import collections
import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libisvd.so")

ISVD_FP64, ISVD_FP32, ISVD_BF16ROT = 0, 1, 2
DTYPE_F32, DTYPE_F64 = 0, 1
ROW, COL, ENTRY = 0, 1, 2
POL_NONE, POL_PERIODIC, POL_ERROR, POL_ANGLE, POL_ADAPTIVE, POL_DRIFT = 0, 1, 2, 3, 4, 5

STATUS = {0: "OK", -1: "E_INVAL", -2: "E_SHAPE", -3: "E_RANGE", -4: "E_NONFINITE", -5: "E_NOMEM",
          -6: "E_BUDGET", -7: "E_DEVICE", -8: "E_STATE", -9: "E_CONVERGE", -10: "E_CAPACITY"}


class IsvdError(RuntimeError):
    def __init__(self, status, where, message):
        super().__init__("%s: %s (%s)" % (where, STATUS.get(status, status), message))
        self.status = status


class CPolicy(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("angle_scope", ctypes.c_int32),
                ("period", ctypes.c_int64), ("check_every", ctypes.c_int64), ("t_min", ctypes.c_int64),
                ("gamma", ctypes.c_double), ("theta_max", ctypes.c_double),
                ("tau", ctypes.c_double), ("band", ctypes.c_double), ("eta", ctypes.c_double),
                ("k_min", ctypes.c_int32), ("k_max", ctypes.c_int32)]


class CConfig(ctypes.Structure):
    _fields_ = [("m0", ctypes.c_int64), ("n0", ctypes.c_int64), ("m_cap", ctypes.c_int64),
                ("n_cap", ctypes.c_int64), ("k", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("tol_rel", ctypes.c_double), ("refresh_iters", ctypes.c_int32),
                ("oversample", ctypes.c_int32), ("policy", CPolicy), ("refresh_tol", ctypes.c_double),
                ("a_on_host", ctypes.c_int32)]


class CMetrics(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("n_refresh", ctypes.c_int64), ("t_last_refresh", ctypes.c_int64),
                ("n_rejected", ctypes.c_int64), ("k", ctypes.c_int32), ("status", ctypes.c_int32),
                ("sweeps", ctypes.c_int32), ("new_direction", ctypes.c_int32)] + [
        (f, ctypes.c_double) for f in ("fro2_A", "sigma2_sum", "evr", "rho", "novelty", "frob_error",
                                       "frob_opt", "frob_gap", "frob_ratio", "ortho_U", "ortho_V",
                                       "update_time_us", "opt_time_us", "angle_ref", "step_angle_U",
                                       "step_angle_V", "spectrum_change")] + [
        ("refresh_rounds", ctypes.c_int32), ("refresh_converged", ctypes.c_int32), ("drift_U", ctypes.c_double), ("angle_opt", ctypes.c_double)]


class CRequest(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("kind", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("payload", ctypes.c_void_p), ("len", ctypes.c_int64), ("i", ctypes.c_int64),
                ("j", ctypes.c_int64), ("delta", ctypes.c_double)]


class CServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_batch", ctypes.c_int32), ("max_inflight", ctypes.c_int32)]


class CCompletion(ctypes.Structure):
    _fields_ = [("req", ctypes.c_int64), ("ticket", ctypes.c_int64), ("kind", ctypes.c_int32),
                ("status", ctypes.c_int32), ("arrival_s", ctypes.c_double), ("admit_s", ctypes.c_double),
                ("launch_s", ctypes.c_double), ("done_s", ctypes.c_double)]


COMPLETION_DTYPE = np.dtype([("req", np.int64), ("ticket", np.int64), ("kind", np.int32), ("status", np.int32),
                             ("arrival_s", np.float64), ("admit_s", np.float64), ("launch_s", np.float64),
                             ("done_s", np.float64)], align=True)
assert COMPLETION_DTYPE.itemsize == ctypes.sizeof(CCompletion)


class CServerStats(ctypes.Structure):
    _fields_ = [("waiting", ctypes.c_int64), ("admitted", ctypes.c_int64), ("retired", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("hbm_used", ctypes.c_uint64), ("inflight_ticks", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("ticks", ctypes.c_int64), ("tick_requests", ctypes.c_int64),
                ("host_admit_s", ctypes.c_double), ("host_tick_s", ctypes.c_double), ("host_wait_s", ctypes.c_double),
                ("host_release_s", ctypes.c_double)]


class CLaunchTime(ctypes.Structure):
    _fields_ = [("phase", ctypes.c_int32), ("kc", ctypes.c_int32), ("fp64", ctypes.c_int32),
                ("nreq", ctypes.c_int32), ("blocks", ctypes.c_int64), ("ms", ctypes.c_double)]


class CRisk(ctypes.Structure):
    _fields_ = [("vol_inc", ctypes.c_double), ("vol_full", ctypes.c_double), ("err_risk", ctypes.c_double),
                ("err_cov", ctypes.c_double)]


# FP32 rotation block shapes: (rows per block, 16-row tiles per wave step, prefetch)
ROT_VARIANTS = [(256, 1, True), (512, 1, True), (1024, 1, True), (1024, 2, False), (2048, 2, False)]

EXPORTS = ["isvd_engine_create", "isvd_engine_destroy", "isvd_stream_bytes", "isvd_init", "isvd_init_from_factors",
           "isvd_append_row", "isvd_append_col", "isvd_update_entry", "isvd_refresh", "isvd_refresh_noalloc", "isvd_metrics",
           "isvd_get_factors", "isvd_get_matrix", "isvd_shape", "isvd_release", "isvd_tick",
           "isvd_profile", "isvd_profile_read", "isvd_autotune", "isvd_set_rotation_variant", "isvd_sync", "isvd_stream_busy", "isvd_rotation_stream", "isvd_set_pipelining", "isvd_set_tick_graphs", "isvd_set_segmented_refresh", "isvd_set_block_cache", "isvd_init_batch",
           "isvd_server_create", "isvd_server_destroy", "isvd_server_clock", "isvd_server_error",
           "isvd_server_add_stream", "isvd_server_submit", "isvd_server_submit_many", "isvd_server_step", "isvd_server_drain",
           "isvd_server_poll", "isvd_server_stats", "isvd_server_stream", "isvd_last_error",
           "isvd_causal_center", "isvd_covariance", "isvd_risk", "isvd_set_deferred_u"]

_lib = None


def load_library(path=LIB_PATH):
    """Load libisvd.so and declare its signatures (no GPU access)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libisvd.so is not built at %s; run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    sig = {
        "isvd_engine_create": (i32, [i32, ctypes.c_uint64, ctypes.POINTER(vp)]),
        "isvd_engine_destroy": (i32, [vp]),
        "isvd_stream_bytes": (ctypes.c_uint64, [ctypes.POINTER(CConfig)]),
        "isvd_init": (i32, [vp, ctypes.POINTER(CConfig), vp, i64, i32, i32, vp, ctypes.POINTER(i64)]),
        "isvd_init_from_factors": (i32, [vp, ctypes.POINTER(CConfig), vp, i64, i32, i32, dp, i64, dp, dp, i64, vp,
                                         ctypes.POINTER(i64)]),
        "isvd_append_row": (i32, [vp, i64, vp, i64, i32, i32, vp]),
        "isvd_append_col": (i32, [vp, i64, vp, i64, i32, i32, vp]),
        "isvd_update_entry": (i32, [vp, i64, i64, i64, ctypes.c_double, vp]),
        "isvd_refresh": (i32, [vp, i64, i32, vp]),
        "isvd_refresh_noalloc": (i32, [vp, i64, i32, vp]),
        "isvd_metrics": (i32, [vp, i64, i32, vp, ctypes.POINTER(CMetrics)]),
        "isvd_causal_center": (i32, [vp, vp, i64, i64, i32, vp, i64, vp]),
        "isvd_covariance": (i32, [vp, i64, vp, i64, vp]),
        "isvd_risk": (i32, [vp, i64, dp, i64, i32, ctypes.POINTER(CRisk), vp]),
        "isvd_get_factors": (i32, [vp, i64, dp, i64, dp, dp, i64, vp]),
        "isvd_get_matrix": (i32, [vp, i64, dp, i64, vp]),
        "isvd_shape": (i32, [vp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32)]),
        "isvd_release": (i32, [vp, i64]),
        "isvd_tick": (i32, [vp, i32, ctypes.POINTER(CRequest), vp]),
        "isvd_profile": (i32, [vp, i32]),
        "isvd_profile_read": (i32, [vp, ctypes.POINTER(CLaunchTime), i32, ctypes.POINTER(i32)]),
        "isvd_autotune": (i32, [vp, vp, ctypes.POINTER(i32), dp]),
        "isvd_set_rotation_variant": (i32, [vp, i32, i32]),
        "isvd_sync": (i32, [vp, vp]),
        "isvd_stream_busy": (i32, [vp, i64, ctypes.POINTER(i32)]),
        "isvd_set_pipelining": (i32, [vp, i32]),
        "isvd_set_tick_graphs": (i32, [vp, i32]),
        "isvd_set_segmented_refresh": (i32, [vp, i32]),
        "isvd_set_block_cache": (i32, [vp, ctypes.c_uint64]),
        "isvd_init_batch": (i32, [vp, i32, ctypes.POINTER(CConfig), ctypes.POINTER(vp), ctypes.POINTER(i64),
                                  ctypes.POINTER(i32), vp, ctypes.POINTER(i64), ctypes.POINTER(i32)]),
        "isvd_set_deferred_u": (i32, [vp, i32, vp]),
        "isvd_server_create": (i32, [vp, ctypes.POINTER(CServerConfig), vp, ctypes.POINTER(vp)]),
        "isvd_server_destroy": (i32, [vp]),
        "isvd_server_clock": (ctypes.c_double, [vp]),
        "isvd_server_error": (ctypes.c_char_p, [vp]),
        "isvd_server_add_stream": (i32, [vp, ctypes.POINTER(CConfig), vp, i64, i32, i64, ctypes.POINTER(i64)]),
        "isvd_server_submit": (i32, [vp, i64, ctypes.POINTER(CRequest), ctypes.c_double, ctypes.POINTER(i64)]),
        "isvd_server_submit_many": (i32, [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(CRequest),
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]),
        "isvd_server_step": (i32, [vp, ctypes.POINTER(i32)]),
        "isvd_server_drain": (i32, [vp]),
        "isvd_server_poll": (i32, [vp, ctypes.POINTER(CCompletion), i32, ctypes.POINTER(i32)]),
        "isvd_server_stats": (i32, [vp, ctypes.POINTER(CServerStats)]),
        "isvd_server_stream": (i32, [vp, i64, ctypes.POINTER(i64), ctypes.POINTER(i32)]),
        "isvd_rotation_stream": (i32, [vp, ctypes.POINTER(vp)]),
        "isvd_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


@dataclass
class Policy:
    kind: int = POL_NONE
    period: int = 0
    check_every: int = 100
    t_min: int = 0
    gamma: float = 1.05
    theta_max: float = 1e-3
    angle_scope: int = 0
    tau: float = 0.95
    band: float = 0.01
    eta: float = 0.5
    k_min: int = 1
    k_max: int = 0

    def to_c(self):
        return CPolicy(self.kind, self.angle_scope, self.period, self.check_every, self.t_min, self.gamma,
                       self.theta_max, self.tau, self.band, self.eta, self.k_min, self.k_max)


def _stream_ptr(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _payload(arr):
    """(pointer, length, dtype code, on_device, keepalive) for numpy or torch input."""
    if hasattr(arr, "data_ptr"):          # torch tensor
        if not arr.is_contiguous():
            raise ValueError("payload tensor must be contiguous")
        dt = str(arr.dtype)
        code = DTYPE_F64 if dt == "torch.float64" else DTYPE_F32 if dt == "torch.float32" else None
        if code is None:
            raise ValueError("payload dtype %s is not float32 / float64" % dt)
        return ctypes.c_void_p(arr.data_ptr()), arr.numel(), code, 1 if arr.is_cuda else 0, arr
    a = np.ascontiguousarray(arr)
    if a.dtype == np.float64:
        code = DTYPE_F64
    elif a.dtype == np.float32:
        code = DTYPE_F32
    else:
        a = a.astype(np.float64)
        code = DTYPE_F64
    return ctypes.c_void_p(a.ctypes.data), a.size, code, 0, a


def causal_center(r, mu, t0, out=None, stream=None):
    """Causal de-meaning (Section 5.1) of the return rows r (device tensor,
    rows x n or n): R_t = r_t - mu_t with the expanding mean mu_t, t = t0 + 1, ...
    mu: device float64 n-vector, the mean after t0 rows on entry (not read
    when t0 = 0), updated in place.  Returns the centred rows (out, or a new
    tensor of r's shape and dtype)."""
    import torch
    lib = load_library()
    if not (hasattr(r, "data_ptr") and r.is_cuda and r.is_contiguous()):
        raise ValueError("r must be a contiguous device tensor")
    if not (hasattr(mu, "data_ptr") and mu.is_cuda and mu.dtype == torch.float64 and mu.is_contiguous()):
        raise ValueError("mu must be a contiguous device float64 tensor")
    n = r.shape[-1]
    rows = r.numel() // n if n else 0
    if mu.numel() != n:
        raise ValueError("mu has %d entries, rows have %d" % (mu.numel(), n))
    if out is None:
        out = torch.empty_like(r)
    code = DTYPE_F64 if r.dtype == torch.float64 else DTYPE_F32 if r.dtype == torch.float32 else None
    if code is None or out.dtype != r.dtype or out.shape != r.shape or not out.is_contiguous():
        raise ValueError("r and out must be float32 / float64 tensors of one shape and dtype")
    st = lib.isvd_causal_center(ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(out.data_ptr()), rows, n, code,
                                ctypes.c_void_p(mu.data_ptr()), int(t0), _stream_ptr(stream))
    if st != 0:
        raise IsvdError(st, "isvd_causal_center", lib.isvd_last_error().decode())
    return out


class Engine:
    """One engine on one HIP device; owns every stream's device state."""

    def __init__(self, device=0, hbm_budget=0):
        self._lib = load_library()
        h = ctypes.c_void_p()
        self._check(self._lib.isvd_engine_create(device, hbm_budget, ctypes.byref(h)), "isvd_engine_create")
        self._h = h

    def _check(self, st, where):
        if st != 0:
            raise IsvdError(st, where, self._lib.isvd_last_error().decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.isvd_engine_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @staticmethod
    def config(m0, n0, k, precision="fp32", m_cap=None, n_cap=None, tol_rel=0.0, policy=None,
               refresh_iters=-1, oversample=-1, refresh_tol=0.0, a_on_host=False):
        prec = {"fp32": ISVD_FP32, "fp64": ISVD_FP64, "bf16rot": ISVD_BF16ROT}[precision]
        pol = (policy or Policy()).to_c()
        return CConfig(m0, n0, m_cap or m0, n_cap or n0, k, prec, tol_rel, refresh_iters, oversample, pol,
                       refresh_tol, 1 if a_on_host else 0)

    def stream_bytes(self, cfg):
        return int(self._lib.isvd_stream_bytes(ctypes.byref(cfg)))

    def init(self, A0, k, precision="fp32", m_cap=None, n_cap=None, tol_rel=0.0, policy=None,
             refresh_iters=-1, oversample=-1, stream=None, refresh_tol=0.0, a_on_host=False):
        if hasattr(A0, "data_ptr"):
            m0, n0 = A0.shape
            ptr, _, code, dev, keep = _payload(A0)
            lda = A0.stride(0)
        else:
            a = np.ascontiguousarray(A0, dtype=np.float64 if np.asarray(A0).dtype != np.float32 else np.float32)
            m0, n0 = a.shape
            ptr, _, code, dev, keep = _payload(a)
            lda = n0
        cfg = self.config(m0, n0, k, precision, m_cap, n_cap, tol_rel, policy, refresh_iters, oversample,
                          refresh_tol, a_on_host)
        sid = ctypes.c_int64()
        self._check(self._lib.isvd_init(self._h, ctypes.byref(cfg), ptr, lda, code, dev, _stream_ptr(stream),
                                        ctypes.byref(sid)), "isvd_init")
        del keep
        return sid.value

    def init_batch(self, A0s, ks, precision="fp32", m_caps=None, n_caps=None, policy=None, refresh_iters=-1,
                   oversample=-1, stream=None):
        """Streams from device tensors A0s (one isvd_init_batch call); returns their ids."""
        n = len(A0s)
        cfgs = (CConfig * n)()
        ptrs = (ctypes.c_void_p * n)()
        ldas = (ctypes.c_int64 * n)()
        dts = (ctypes.c_int32 * n)()
        keep = []
        for q, A0 in enumerate(A0s):
            m0, n0 = A0.shape
            ptr, _, code, dev, k = _payload(A0)
            if not dev:
                raise ValueError("init_batch takes device tensors")
            keep.append(k)
            cfgs[q] = self.config(m0, n0, ks[q], precision, m_caps[q] if m_caps else None,
                                  n_caps[q] if n_caps else None, 0.0, policy, refresh_iters, oversample)
            ptrs[q] = ptr
            ldas[q] = A0.stride(0)
            dts[q] = code
        ids = (ctypes.c_int64 * n)()
        made = ctypes.c_int32()
        self._check(self._lib.isvd_init_batch(self._h, n, cfgs, ptrs, ldas, dts, _stream_ptr(stream), ids,
                                              ctypes.byref(made)), "isvd_init_batch")
        return [ids[q] for q in range(n)]

    def init_from_factors(self, A0, U, S, V, precision="fp32", m_cap=None, n_cap=None, tol_rel=0.0, policy=None,
                          refresh_iters=-1, oversample=-1, stream=None, refresh_tol=0.0):
        """Start a stream from given FP64 factors (U m0 x k, S k, V n0 x k) and A0."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        S = np.ascontiguousarray(S, dtype=np.float64)
        V = np.ascontiguousarray(V, dtype=np.float64)
        k = S.shape[0]
        if hasattr(A0, "data_ptr"):
            m0, n0 = A0.shape
            ptr, _, code, dev, keep = _payload(A0)
            lda = A0.stride(0)
        else:
            a = np.ascontiguousarray(A0, dtype=np.float64 if np.asarray(A0).dtype != np.float32 else np.float32)
            m0, n0 = a.shape
            ptr, _, code, dev, keep = _payload(a)
            lda = n0
        cfg = self.config(m0, n0, k, precision, m_cap, n_cap, tol_rel, policy, refresh_iters, oversample,
                          refresh_tol)
        sid = ctypes.c_int64()
        dp = ctypes.POINTER(ctypes.c_double)
        self._check(self._lib.isvd_init_from_factors(self._h, ctypes.byref(cfg), ptr, lda, code, dev,
                                                     U.ctypes.data_as(dp), k, S.ctypes.data_as(dp),
                                                     V.ctypes.data_as(dp), k, _stream_ptr(stream),
                                                     ctypes.byref(sid)), "isvd_init_from_factors")
        del keep
        return sid.value

    def append_row(self, sid, x, stream=None):
        ptr, n, code, dev, keep = _payload(x)
        self._check(self._lib.isvd_append_row(self._h, sid, ptr, n, code, dev, _stream_ptr(stream)),
                    "isvd_append_row")

    def append_col(self, sid, y, stream=None):
        ptr, m, code, dev, keep = _payload(y)
        self._check(self._lib.isvd_append_col(self._h, sid, ptr, m, code, dev, _stream_ptr(stream)),
                    "isvd_append_col")

    def update_entry(self, sid, i, j, delta, stream=None):
        self._check(self._lib.isvd_update_entry(self._h, sid, int(i), int(j), float(delta), _stream_ptr(stream)),
                    "isvd_update_entry")

    def refresh(self, sid, store_reference=True, stream=None):
        self._check(self._lib.isvd_refresh(self._h, sid, 1 if store_reference else 0, _stream_ptr(stream)),
                    "isvd_refresh")

    def refresh_noalloc(self, sid, store_reference=True, stream=None):
        """isvd_refresh with its workspace in the library's static device array
        (no device allocation)."""
        self._check(self._lib.isvd_refresh_noalloc(self._h, sid, 1 if store_reference else 0, _stream_ptr(stream)),
                    "isvd_refresh_noalloc")

    def metrics(self, sid, exact=False, stream=None):
        out = CMetrics()
        self._check(self._lib.isvd_metrics(self._h, sid, 1 if exact else 0, _stream_ptr(stream), ctypes.byref(out)),
                    "isvd_metrics")
        return {f: getattr(out, f) for f, _ in CMetrics._fields_}

    def covariance(self, sid, out=None, stream=None):
        """Low-rank covariance V diag(sigma^2) V^T / (m - 1) of the stream
        (Section 5.3) as an n x n float64 device tensor."""
        import torch
        _, n, _ = self.shape(sid)
        if out is None:
            out = torch.empty((n, n), dtype=torch.float64, device="cuda")
        if out.dtype != torch.float64 or not out.is_cuda or out.dim() != 2 or out.stride(1) != 1:
            raise ValueError("out must be a row-major float64 device matrix")
        self._check(self._lib.isvd_covariance(self._h, sid, ctypes.c_void_p(out.data_ptr()), out.stride(0),
                                              _stream_ptr(stream)), "isvd_covariance")
        return out

    def risk(self, sid, w, exact=False, stream=None):
        """Portfolio volatility of weights w (Section 5.3); with exact also the
        truncated SVD's volatility, the risk error and the covariance error."""
        w = np.ascontiguousarray(w, dtype=np.float64)
        out = CRisk()
        dp = ctypes.POINTER(ctypes.c_double)
        self._check(self._lib.isvd_risk(self._h, sid, w.ctypes.data_as(dp), w.size, 1 if exact else 0,
                                        ctypes.byref(out), _stream_ptr(stream)), "isvd_risk")
        return {f: getattr(out, f) for f, _ in CRisk._fields_}

    def shape(self, sid):
        m, n, k = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        self._check(self._lib.isvd_shape(self._h, sid, ctypes.byref(m), ctypes.byref(n), ctypes.byref(k)),
                    "isvd_shape")
        return m.value, n.value, k.value

    def factors(self, sid, stream=None):
        met = self.metrics(sid, stream=stream)
        m, n, k = met["m"], met["n"], met["k"]
        U = np.zeros((m, k))
        S = np.zeros(k)
        V = np.zeros((n, k))
        dp = ctypes.POINTER(ctypes.c_double)
        self._check(self._lib.isvd_get_factors(self._h, sid, U.ctypes.data_as(dp), max(k, 1), S.ctypes.data_as(dp),
                                               V.ctypes.data_as(dp), max(k, 1), _stream_ptr(stream)),
                    "isvd_get_factors")
        return U, S, V

    def matrix(self, sid, stream=None):
        m, n, _ = self.shape(sid)
        A = np.zeros((m, n))
        self._check(self._lib.isvd_get_matrix(self._h, sid, A.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n,
                                              _stream_ptr(stream)), "isvd_get_matrix")
        return A

    def release(self, sid):
        self._check(self._lib.isvd_release(self._h, sid), "isvd_release")

    def tick(self, requests, stream=None):
        """requests: list of (sid, kind, payload tensor) or (sid, ENTRY, (i, j, delta))."""
        arr = (CRequest * len(requests))()
        keep = []
        for q, (sid, kind, pay) in enumerate(requests):
            r = arr[q]
            r.id = sid
            r.kind = kind
            if kind == ENTRY:
                r.i, r.j, r.delta = int(pay[0]), int(pay[1]), float(pay[2])
                r.dtype = DTYPE_F32
            else:
                ptr, ln, code, dev, k = _payload(pay)
                if not dev:
                    raise ValueError("tick payloads must be device tensors")
                keep.append(k)
                r.payload = ptr
                r.len = ln
                r.dtype = code
        self._check(self._lib.isvd_tick(self._h, len(requests), arr, _stream_ptr(stream)), "isvd_tick")

    @staticmethod
    def tick_requests(requests):
        """Pre-marshalled request array for repeated ticks (bench loops)."""
        arr = (CRequest * len(requests))()
        for q, (sid, kind, pay) in enumerate(requests):
            arr[q].id = sid
            arr[q].kind = kind
            if kind == ENTRY:
                arr[q].i, arr[q].j, arr[q].delta = int(pay[0]), int(pay[1]), float(pay[2])
            else:
                arr[q].payload = ctypes.c_void_p(pay.data_ptr())
                arr[q].len = pay.numel()
                arr[q].dtype = DTYPE_F64 if str(pay.dtype) == "torch.float64" else DTYPE_F32
        return arr

    def profile(self, enable=True):
        self._check(self._lib.isvd_profile(self._h, 1 if enable else 0), "isvd_profile")

    def profile_read(self):
        cnt = ctypes.c_int32()
        self._check(self._lib.isvd_profile_read(self._h, None, 0, ctypes.byref(cnt)), "isvd_profile_read")
        arr = (CLaunchTime * max(cnt.value, 1))()
        self._check(self._lib.isvd_profile_read(self._h, arr, cnt.value, ctypes.byref(cnt)), "isvd_profile_read")
        return [{f: getattr(arr[q], f) for f, _ in CLaunchTime._fields_} for q in range(cnt.value)]

    def autotune(self, stream=None):
        """Time the FP32 rotation's block shapes per rank bucket and keep the
        fastest.  Returns {bucket: (variant chosen, [ms per launch of each variant])};
        ROT_VARIANTS lists the shapes."""
        var = (ctypes.c_int32 * 4)()
        ms = (ctypes.c_double * (4 * len(ROT_VARIANTS)))()
        self._check(self._lib.isvd_autotune(self._h, _stream_ptr(stream), var, ms), "isvd_autotune")
        nv = len(ROT_VARIANTS)
        return {kc: (var[b], [ms[nv * b + c] for c in range(nv)]) for b, kc in enumerate((8, 16, 32, 64))}

    def set_rotation_variant(self, kc, variant):
        self._check(self._lib.isvd_set_rotation_variant(self._h, kc, variant), "isvd_set_rotation_variant")

    def sync(self, stream=None):
        """Order `stream` after the U rotations still pending from pipelined ticks
        and the refreshes still running on the refresh lanes."""
        self._check(self._lib.isvd_sync(self._h, _stream_ptr(stream)), "isvd_sync")

    def busy(self, sid):
        """True while a refresh fired by a tick still runs for stream `sid`."""
        out = ctypes.c_int32(0)
        self._check(self._lib.isvd_stream_busy(self._h, sid, ctypes.byref(out)), "isvd_stream_busy")
        return bool(out.value)

    def set_pipelining(self, enable):
        self._check(self._lib.isvd_set_pipelining(self._h, 1 if enable else 0), "isvd_set_pipelining")

    def set_block_cache(self, nbytes):
        """Keep released streams' device blocks (up to nbytes) for later
        streams (see isvd_set_block_cache in include/isvd.h)."""
        self._check(self._lib.isvd_set_block_cache(self._h, int(nbytes)), "isvd_set_block_cache")

    def set_segmented_refresh(self, enable):
        """Compute the refreshes one tick fires as one segmented batch (see
        isvd_set_segmented_refresh in include/isvd.h)."""
        self._check(self._lib.isvd_set_segmented_refresh(self._h, 1 if enable else 0), "isvd_set_segmented_refresh")

    def set_tick_graphs(self, enable):
        """Replay deferred-U row-append ticks as captured HIP graphs."""
        self._check(self._lib.isvd_set_tick_graphs(self._h, 1 if enable else 0), "isvd_set_tick_graphs")

    def set_deferred_u(self, enable, stream=None):
        """Brand's deferred left basis U = U0 W for the row appends of eligible
        streams (see isvd_set_deferred_u in include/isvd.h)."""
        self._check(self._lib.isvd_set_deferred_u(self._h, 1 if enable else 0, _stream_ptr(stream)),
                    "isvd_set_deferred_u")

    def rotation_stream(self):
        """Handle (int) of the engine's rotation stream.  A tick's updates are
        done once both the caller's stream and this stream have passed it
        (wrap it with torch.cuda.ExternalStream and record an event on each)."""
        out = ctypes.c_void_p()
        self._check(self._lib.isvd_rotation_stream(self._h, ctypes.byref(out)), "isvd_rotation_stream")
        return out.value or 0

    def tick_raw(self, arr, stream=None):
        self._check(self._lib.isvd_tick(self._h, len(arr), arr, _stream_ptr(stream)), "isvd_tick")


class Server:
    """Serving loop over an Engine (continuous batching, HBM-budget admission);
    scheduling runs in the library (isvd_server_*)."""

    def __init__(self, engine, hbm_budget=0, max_batch=0, max_inflight=2, stream=None):
        self._eng = engine
        self._lib = engine._lib
        cfg = CServerConfig(int(hbm_budget), int(max_batch), int(max_inflight))
        h = ctypes.c_void_p()
        self._check(self._lib.isvd_server_create(engine._h, ctypes.byref(cfg), _stream_ptr(stream), ctypes.byref(h)),
                    "isvd_server_create")
        self._h = h
        self._keep = {}
        self._pending = collections.deque()   # tickets whose A0 is held, in admission (FIFO) order

    def _check(self, st, where):
        if st != 0:
            msg = self._lib.isvd_server_error(self._h).decode() if getattr(self, "_h", None) else ""
            raise IsvdError(st, where, msg or self._lib.isvd_last_error().decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.isvd_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def clock(self):
        return float(self._lib.isvd_server_clock(self._h))

    def add_stream(self, A0, k, precision="fp32", m_cap=None, n_cap=None, lifetime=0, policy=None, tol_rel=0.0,
                   refresh_iters=-1, oversample=-1):
        """A0: a device tensor kept alive by the server until the stream is
        admitted (admission copies it on the server's stream; allocate it on
        that stream so that its memory is reused only after the copy)."""
        m0, n0 = A0.shape
        ptr, _, code, dev, keep = _payload(A0)
        if not dev:
            raise ValueError("A0 must be a device tensor")
        cfg = Engine.config(m0, n0, k, precision, m_cap, n_cap, tol_rel, policy, refresh_iters, oversample)
        t = ctypes.c_int64()
        self._check(self._lib.isvd_server_add_stream(self._h, ctypes.byref(cfg), ptr, A0.stride(0), code,
                                                     int(lifetime), ctypes.byref(t)), "isvd_server_add_stream")
        self._keep[("A0", t.value)] = keep
        self._pending.append(t.value)
        return t.value

    def submit(self, ticket, kind, payload, arrival_s):
        """payload: device tensor (row / column) or (i, j, delta) for an entry update."""
        r = CRequest()
        r.kind = kind
        if kind == ENTRY:
            r.i, r.j, r.delta = int(payload[0]), int(payload[1]), float(payload[2])
            r.dtype = DTYPE_F32
        else:
            ptr, ln, code, dev, keep = _payload(payload)
            if not dev:
                raise ValueError("payloads must be device tensors")
            r.payload = ptr
            r.len = ln
            r.dtype = code
        rid = ctypes.c_int64()
        self._check(self._lib.isvd_server_submit(self._h, int(ticket), ctypes.byref(r), float(arrival_s),
                                                 ctypes.byref(rid)), "isvd_server_submit")
        if kind != ENTRY:
            self._keep[rid.value] = keep
        return rid.value

    def submit_many(self, tickets, reqs, arrivals):
        """tickets: int64 array, reqs: a CRequest array (payloads kept alive by the
        caller until completion), arrivals: float64 array."""
        t = np.ascontiguousarray(tickets, dtype=np.int64)
        a = np.ascontiguousarray(arrivals, dtype=np.float64)
        n = len(t)
        if n == 0:
            return
        self._check(self._lib.isvd_server_submit_many(
            self._h, n, t.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), reqs,
            a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None), "isvd_server_submit_many")

    def step(self):
        n = ctypes.c_int32()
        self._check(self._lib.isvd_server_step(self._h, ctypes.byref(n)), "isvd_server_step")
        # admission is FIFO: release the A0 of the admitted head of the queue
        while self._pending and self.stream(self._pending[0])[1] != 0:
            self._keep.pop(("A0", self._pending.popleft()), None)
        return n.value

    def held_a0(self):
        """Streams whose A0 the server still holds (not yet admitted)."""
        return len(self._pending)

    def drain(self):
        self._check(self._lib.isvd_server_drain(self._h), "isvd_server_drain")

    def poll(self, cap=1 << 16):
        arr = (CCompletion * cap)()
        n = ctypes.c_int32()
        self._check(self._lib.isvd_server_poll(self._h, arr, cap, ctypes.byref(n)), "isvd_server_poll")
        out = [{f: getattr(arr[q], f) for f, _ in CCompletion._fields_} for q in range(n.value)]
        for c in out:
            self._keep.pop(c["req"], None)
        return out

    def poll_array(self, cap=1 << 16):
        """Completion records as a numpy structured array (COMPLETION_DTYPE),
        oldest first."""
        if getattr(self, "_pbuf", None) is None or len(self._pbuf) < cap:
            self._pbuf = (CCompletion * cap)()
        arr = self._pbuf
        n = ctypes.c_int32()
        self._check(self._lib.isvd_server_poll(self._h, arr, cap, ctypes.byref(n)), "isvd_server_poll")
        out = np.frombuffer(arr, dtype=COMPLETION_DTYPE, count=n.value).copy()
        if len(self._keep) > len(self._pending):
            for rid in out["req"].tolist():
                self._keep.pop(rid, None)
        return out

    def stats(self):
        st = CServerStats()
        self._check(self._lib.isvd_server_stats(self._h, ctypes.byref(st)), "isvd_server_stats")
        return {f: getattr(st, f) for f, _ in CServerStats._fields_ if f != "pad"}

    def stream(self, ticket):
        sid, state = ctypes.c_int64(), ctypes.c_int32()
        self._check(self._lib.isvd_server_stream(self._h, int(ticket), ctypes.byref(sid), ctypes.byref(state)),
                    "isvd_server_stream")
        return sid.value, state.value
