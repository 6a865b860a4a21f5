"""Oracle full and truncated SVD (FP64), via the C one-sided Jacobi routine.

Background section of the paper: A = U Sigma V^T with non-increasing
singular values; the truncated SVD of rank k keeps the leading k triplets,
and by Eckart-Young ||A - A_k||_F^2 is the sum of the trailing sigma_i^2.
"""
import ctypes

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        lib.oracle_jacobi_svd.restype = ctypes.c_int
        i64 = ctypes.c_int64
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_jacobi_svd.argtypes = [i64, i64, dp, i64, dp, i64, dp, dp, i64, ctypes.c_int]
        _lib = lib
    return _lib


class JacobiNotConverged(RuntimeError):
    pass


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def svd(A, max_sweeps=60):
    """Thin SVD (U, s, V) of any real matrix: A = U diag(s) V^T.

    For m >= n, U is m x n and V is n x n; for m < n the routine runs on A^T
    and swaps the roles, so U is m x m and V is n x m."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        V, s, U = svd(A.T, max_sweeps)
        return U, s, V
    U = np.zeros((m, n))
    V = np.zeros((n, n))
    s = np.zeros(n)
    rc = _load().oracle_jacobi_svd(m, n, _ptr(A), n, _ptr(U), n, _ptr(s), _ptr(V), n, max_sweeps)
    if rc == -1:
        raise JacobiNotConverged("one-sided Jacobi hit %d sweeps" % max_sweeps)
    if rc < 0:
        raise ValueError("oracle_jacobi_svd: bad arguments")
    return U, s, V


# Singular values at or below RANK_TOL * sigma_1 count as zero: a matrix whose
# spectrum ends there has that numerical rank, and TruncatedSVD(A, k) keeps
# min(k, numerical rank) triplets (the directions past it are arbitrary at
# FP64 rounding).  The engine's refresh uses the same threshold.
RANK_TOL = 1e-12


def truncated_svd(A, k):
    """TruncatedSVD(A, k) (Sec. 2.4.1): the leading min(k, numerical rank)
    triplets, sigma > RANK_TOL * sigma_1."""
    U, s, V = svd(A)
    r = int(min(k, np.count_nonzero(s > RANK_TOL * (s[0] if s.size else 0.0)))) if s.size and s[0] > 0 else 0
    return U[:, :r].copy(), s[:r].copy(), V[:, :r].copy()


def singular_values(A):
    return svd(A)[1]
