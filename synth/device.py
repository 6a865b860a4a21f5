"""Device-side factor-model rows (same entries as FactorStream, generated in HBM).

Inputs only.  Used where the host generator would be too slow (tens of GB of
panels); ``tests/test_synth_device.py`` checks it against the numpy path.
"""
import ctypes
import os
import subprocess

import numpy as np

from .factor_model import factor_lambdas

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "synth.hip")
LIB = os.path.join(HERE, "libsynth.so")

_lib = None


def build(force=True):
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", SRC, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError("libsynth.so not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB)
        lib.synth_rows.restype = ctypes.c_int
        lib.synth_rows.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_void_p]
        lib.synth_rows_async.restype = ctypes.c_int
        lib.synth_rows_async.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                         ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def _out_dtype(out, rows, cols, ld):
    """dtype code of the device tensor `out` after checking that rows x cols
    entries at leading dimension ld lie inside its storage."""
    if str(out.dtype) not in ("torch.float32", "torch.float64"):
        raise TypeError("out must be float32 or float64")
    if not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous device tensor")
    if rows < 0 or cols < 0 or ld < cols or (rows > 0 and (rows - 1) * ld + cols > out.numel()):
        raise ValueError("rows x cols at leading dimension %d do not fit in out" % ld)
    return 1 if str(out.dtype) == "torch.float64" else 0


def rows_into(out, row0, rows, cols, seed, stream, K, noise=0.1, lambdas=None, ld=None, hip_stream=None):
    """Fill the device tensor `out` (rows x cols, leading dim ld) with rows
    [row0, row0 + rows) of the (seed, stream) panel."""
    lam = np.ascontiguousarray(lambdas if lambdas is not None else factor_lambdas(K), dtype=np.float64)
    dtype = _out_dtype(out, rows, cols, ld or cols)
    rc = _load().synth_rows(ctypes.c_void_p(out.data_ptr()), ld or cols, dtype, row0, rows, cols, seed, stream, K,
                            lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), noise,
                            ctypes.c_void_p(hip_stream) if hip_stream else None)
    if rc != 0:
        raise RuntimeError("synth_rows failed with HIP error %d" % rc)
    return out


class AsyncRows:
    """Device rows of panels with at most max_rows x max_cols entries,
    queued on one HIP stream without allocating or waiting (the buffers are
    reused in that stream's order)."""

    def __init__(self, max_rows, max_cols, K, lambdas=None, device="cuda"):
        import torch
        self.K = K
        lam = np.ascontiguousarray(lambdas if lambdas is not None else factor_lambdas(K), dtype=np.float64)
        self.L = torch.tensor(lam, dtype=torch.float64, device=device)
        self.F = torch.empty(max_rows * K, dtype=torch.float64, device=device)
        self.B = torch.empty(max_cols * K, dtype=torch.float64, device=device)
        self.max_rows, self.max_cols = max_rows, max_cols

    def rows_into(self, out, row0, rows, cols, seed, stream, hip_stream, noise=0.1, ld=None):
        if rows > self.max_rows or cols > self.max_cols:
            raise ValueError("panel larger than the buffers")
        dtype = _out_dtype(out, rows, cols, ld or cols)
        rc = _load().synth_rows_async(ctypes.c_void_p(out.data_ptr()), ld or cols, dtype, row0, rows, cols, seed,
                                      stream, self.K, ctypes.c_void_p(self.L.data_ptr()), noise,
                                      ctypes.c_void_p(self.F.data_ptr()), ctypes.c_void_p(self.B.data_ptr()),
                                      ctypes.c_void_p(hip_stream))
        if rc != 0:
            raise RuntimeError("synth_rows_async failed with HIP error %d" % rc)
        return out
