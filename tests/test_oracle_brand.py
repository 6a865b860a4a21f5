"""Pins of the oracle's Brand updates against what the paper and linear algebra fix.

* untruncated row / column appends equal the SVD of the appended matrix
  (the block derivation of Section 2.2.1 is exact);
* truncated appends equal the best rank-k approximation of [A_hat; x^T]
  (exact up to rank-k truncation, Section 3 opening);
* the rho <= tol branch keeps the rank and the result;
* column append = row append on the transpose (Algorithm A2), bitwise;
* the rank-1 update satisfies eq. rank1-projection:
  U' S' V'^T = P_U (A_hat + delta e_i e_j^T) P_V, and keeps span(U), span(V).

The last tests plant plausible mistakes into copies of the oracle's update
(a transposed core factor, a dropped rho, a column of V instead of a row, a
wrong sign) and check that the pins above reject each of them."""
import numpy as np
import pytest

from oracle import brand
from oracle.svd import svd, truncated_svd


def _lapack_best_rank_k(M, k):
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    return (U[:, :k] * s[:k]) @ Vt[:k]


def _recon(U, s, V):
    return (U * s) @ V.T


def _state(rng, m, n, k):
    A = rng.standard_normal((m, n))
    U, s, V = truncated_svd(A, k)
    return U, s, V


@pytest.mark.parametrize("cgs2", [False, True])
def test_row_append_untruncated_equals_svd_of_appended(cgs2):
    rng = np.random.default_rng(0)
    m, n = 8, 12                         # m < n: every new row brings a new direction
    A = rng.standard_normal((m, n))
    U, s, V = svd(A)                     # exact, r = m
    x = rng.standard_normal(n)
    U2, s2, V2, info = brand.row_append(U, s, V, x, k_keep=m + 1, cgs2=cgs2)
    M = np.vstack([A, x])
    assert info.new_direction and len(s2) == m + 1
    s_ref = np.linalg.svd(M, compute_uv=False)
    assert np.max(np.abs(s2 - s_ref)) <= 1e-12 * s_ref[0]
    assert np.linalg.norm(_recon(U2, s2, V2) - M) <= 1e-12 * np.linalg.norm(M)
    assert np.linalg.norm(U2.T @ U2 - np.eye(m + 1)) < 1e-12
    assert np.linalg.norm(V2.T @ V2 - np.eye(m + 1)) < 1e-12


def test_row_append_rho_below_tol_keeps_rank():
    rng = np.random.default_rng(1)
    m, n = 12, 6                         # n <= k: x is always in span(V)
    A = rng.standard_normal((m, n))
    U, s, V = svd(A)
    x = rng.standard_normal(n)
    U2, s2, V2, info = brand.row_append(U, s, V, x, k_keep=10)
    assert not info.new_direction and info.rho == 0.0
    assert len(s2) == n                  # sigma' = 0 is never kept
    M = np.vstack([A, x])
    assert np.max(np.abs(s2 - np.linalg.svd(M, compute_uv=False))) <= 1e-12 * s2[0]
    assert np.linalg.norm(_recon(U2, s2, V2) - M) <= 1e-12 * np.linalg.norm(M)
    assert np.linalg.norm(V2.T @ V2 - np.eye(n)) < 1e-12


@pytest.mark.parametrize("m,n,k", [(30, 20, 5), (60, 40, 12), (25, 25, 24)])
def test_row_append_truncated_equals_best_rank_k(m, n, k):
    rng = np.random.default_rng(m + n + k)
    U, s, V = _state(rng, m, n, k)
    x = rng.standard_normal(n) * 2.0
    U2, s2, V2, _ = brand.row_append(U, s, V, x, k_keep=k)
    M = np.vstack([_recon(U, s, V), x])
    ref = _lapack_best_rank_k(M, k)
    assert np.linalg.norm(_recon(U2, s2, V2) - ref) <= 1e-12 * np.linalg.norm(ref)


def test_col_append_is_row_append_on_transpose():
    rng = np.random.default_rng(2)
    U, s, V = _state(rng, 30, 20, 6)
    y = rng.standard_normal(30)
    U2, s2, V2, _ = brand.col_append(U, s, V, y, k_keep=6)
    Vt, st, Ut, _ = brand.row_append(V, s, U, y, k_keep=6)
    assert np.array_equal(U2, Ut) and np.array_equal(s2, st) and np.array_equal(V2, Vt)
    M = np.hstack([_recon(U, s, V), y[:, None]])
    ref = _lapack_best_rank_k(M, 6)
    assert np.linalg.norm(_recon(U2, s2, V2) - ref) <= 1e-12 * np.linalg.norm(ref)


def test_rank_one_projection_identity():
    rng = np.random.default_rng(3)
    m, n, k = 40, 25, 7
    U, s, V = _state(rng, m, n, k)
    Ahat = _recon(U, s, V)
    for (i, j, d) in [(0, 0, 0.7), (39, 24, -1.3), (17, 3, 5.0)]:
        U2, s2, V2 = brand.rank_one(U, s, V, i, j, d)
        E = np.zeros((m, n))
        E[i, j] = d
        PU = U @ U.T
        PV = V @ V.T
        target = PU @ (Ahat + E) @ PV
        assert np.linalg.norm(_recon(U2, s2, V2) - target) <= 1e-13 * np.linalg.norm(target)
        # span(U') = span(U), span(V') = span(V): all principal cosines are 1
        assert np.max(np.abs(np.linalg.svd(U.T @ U2, compute_uv=False) - 1.0)) < 1e-13
        assert np.max(np.abs(np.linalg.svd(V.T @ V2, compute_uv=False) - 1.0)) < 1e-13
        assert np.all(np.diff(s2) <= 0) and len(s2) == k


# --------------------------------------------------------------- planted mistakes
def _row_append_variant(U, s, V, x, k_keep, mistake):
    m, r = U.shape
    p = V.T @ x
    z = x - V @ p
    rho = np.linalg.norm(z)
    zhat = z / rho
    K = np.zeros((r + 1, r + 1))
    K[:r, :r] = np.diag(s)
    K[r, :r] = -p if mistake == "sign" else p
    K[r, r] = 0.0 if mistake == "drop_rho" else rho
    UK, sK, VK = svd(K)
    Ulift = np.zeros((m + 1, r + 1))
    Ulift[:m, :r] = U
    Ulift[m, r] = 1.0
    Un = Ulift @ UK
    Vn = np.hstack([V, zhat[:, None]]) @ (VK.T if mistake == "transpose" else VK)
    return Un[:, :k_keep], sK[:k_keep], Vn[:, :k_keep]


@pytest.mark.parametrize("mistake", ["sign", "drop_rho", "transpose"])
def test_pins_reject_planted_row_append_mistakes(mistake):
    rng = np.random.default_rng(4)
    U, s, V = _state(rng, 30, 20, 5)
    x = rng.standard_normal(20) * 3.0
    M = np.vstack([_recon(U, s, V), x])
    ref = _lapack_best_rank_k(M, 5)
    U2, s2, V2 = _row_append_variant(U, s, V, x, 5, mistake)
    assert np.linalg.norm(_recon(U2, s2, V2) - ref) > 1e-6 * np.linalg.norm(ref)
    U3, s3, V3 = _row_append_variant(U, s, V, x, 5, None)
    assert np.linalg.norm(_recon(U3, s3, V3) - ref) <= 1e-12 * np.linalg.norm(ref)


def test_pins_reject_rank_one_with_column_of_V():
    rng = np.random.default_rng(5)
    m, n, k = 30, 20, 6
    U, s, V = _state(rng, m, n, k)
    i, j, d = 4, 2, 1.5
    su, sv_wrong = U[i, :], V[:k, j]     # column j of V instead of row j
    K = np.diag(s) + d * np.outer(su, sv_wrong)
    UK, sK, VK = svd(K)
    E = np.zeros((m, n))
    E[i, j] = d
    target = U @ U.T @ (_recon(U, s, V) + E) @ V @ V.T
    got = ((U @ UK) * sK) @ (V @ VK).T
    assert np.linalg.norm(got - target) > 1e-6 * np.linalg.norm(target)
