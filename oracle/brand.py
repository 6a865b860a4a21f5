"""Oracle Brand-style updates (FP64), in the paper's order and notation.

Row append (Section 2.2.1, Algorithm A1), column append via the transpose
(Section 2.2.2, Algorithm A2) and the rank-1 entry update (Section 2.3,
Algorithm A3), each followed by the truncation of the engine loop
(Algorithm 1).  The small core SVD is the oracle's own Jacobi routine.

Readings of points the paper leaves open:
* tol: a new direction counts iff rho > tol with tol = tol_rel * ||x||; when
  it does not, both z_hat and rho are taken as zero in the core (Section
  2.2.1 treats rho <= tol as zero; Algorithm A1 zeroes z_hat only -- the
  reconstruction is the same either way, zeroing rho keeps V' orthonormal).
* truncation keeps min(k_keep, r + 1) triplets but never a triplet whose
  singular value is exactly zero (no rank growth when x lies in span V).
* s_v of the rank-1 update is the j-th *row* of V (column j of V^T), as in
  Algorithm A3.
* ``cgs2`` adds one re-orthogonalisation pass to the projection of the new
  row (classical Gram-Schmidt twice); the paper projects once.  In FP64 the
  two agree to rounding.
"""
from dataclasses import dataclass

import numpy as np

from .svd import svd


@dataclass
class AppendInfo:
    p: np.ndarray          # coordinates of the new row in span(V)
    rho: float             # residual norm ||z|| (0 if below tol)
    xnorm: float           # ||x||
    new_direction: bool    # rho > tol
    sigma_dropped: float   # largest singular value removed by truncation (0 if none)


def _keep_count(s_new, k_keep):
    r = min(int(k_keep), len(s_new))
    while r > 0 and s_new[r - 1] == 0.0:
        r -= 1
    return r


def row_append(U, s, V, x, k_keep, tol_rel=1e-10, cgs2=False):
    """Algorithm A1 then truncation to k_keep.  Returns (U', s', V', info)."""
    x = np.asarray(x, dtype=np.float64)
    m, r = U.shape
    # Step 1: projection onto the current right-singular subspace
    p = V.T @ x
    z = x - V @ p
    if cgs2:
        p2 = V.T @ z
        z = z - V @ p2
        p = p + p2
    rho = float(np.linalg.norm(z))
    xnorm = float(np.linalg.norm(x))
    new_dir = rho > tol_rel * xnorm
    if new_dir:
        zhat = z / rho
    else:
        zhat = np.zeros_like(z)
        rho = 0.0
    # Step 2: small core SVD of K = [[Sigma, 0], [p, rho]]
    K = np.zeros((r + 1, r + 1))
    K[:r, :r] = np.diag(s)
    K[r, :r] = p
    K[r, r] = rho
    UK, sK, VK = svd(K)
    # Step 3: lift the core's singular vectors
    Ulift = np.zeros((m + 1, r + 1))
    Ulift[:m, :r] = U
    Ulift[m, r] = 1.0
    U_new = Ulift @ UK
    V_new = np.hstack([V, zhat[:, None]]) @ VK
    keep = _keep_count(sK, k_keep)
    dropped = float(sK[keep]) if keep < len(sK) else 0.0
    info = AppendInfo(p=p, rho=rho, xnorm=xnorm, new_direction=new_dir, sigma_dropped=dropped)
    return U_new[:, :keep], sK[:keep], V_new[:, :keep], info


def col_append(U, s, V, y, k_keep, tol_rel=1e-10, cgs2=False):
    """Algorithm A2: a row append on the transpose, then swap back."""
    Vt_new, s_new, Ut_new, info = row_append(V, s, U, y, k_keep, tol_rel, cgs2)
    return Ut_new, s_new, Vt_new, info


def rank_one(U, s, V, i, j, delta):
    """Algorithm A3: K = Sigma + delta s_u s_v^T, U' = U U_K, V' = V V_K.

    The rank is preserved (no truncation is needed)."""
    su = U[i, :]
    sv = V[j, :]
    K = np.diag(s) + delta * np.outer(su, sv)
    UK, sK, VK = svd(K)
    return U @ UK, sK, V @ VK


def truncate(U, s, V, k):
    r = _keep_count(s, k)
    return U[:, :r], s[:r], V[:, :r]
