"""Pins of the oracle's own one-sided Jacobi SVD (FP64).

Against: LAPACK (numpy.linalg.svd), the 2x2 closed form, diagonal / zero /
rank-deficient / repeated-singular-value special cases, Eckart-Young."""
import numpy as np
import pytest

from oracle.svd import svd, truncated_svd

EPS = np.finfo(np.float64).eps


def _check_factorisation(A, U, s, V, tol=1e-13):
    scale = max(np.linalg.norm(A), 1e-300)
    assert np.linalg.norm(A - (U * s) @ V.T) <= tol * scale * max(A.shape)
    assert np.all(np.diff(s) <= 0.0)
    assert np.all(s >= 0.0)
    r = np.count_nonzero(s > 0)
    assert np.linalg.norm(U[:, :r].T @ U[:, :r] - np.eye(r)) <= tol * max(A.shape)
    assert np.linalg.norm(V.T @ V - np.eye(V.shape[1])) <= tol * max(A.shape)


@pytest.mark.parametrize("m,n,seed", [(7, 7, 0), (40, 12, 1), (300, 50, 2), (12, 40, 3), (1, 1, 4), (5, 1, 5)])
def test_matches_lapack_on_random(m, n, seed):
    A = np.random.default_rng(seed).standard_normal((m, n))
    U, s, V = svd(A)
    _check_factorisation(A, U, s, V)
    s_ref = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(s - s_ref)) <= 1e-13 * s_ref[0]
    # singular subspaces of well separated values agree with LAPACK's
    Ur, sr, Vrt = np.linalg.svd(A, full_matrices=False)
    for i in range(min(m, n)):
        gap = min([abs(sr[i] - sr[j]) for j in range(len(sr)) if j != i] + [np.inf])
        if gap > 1e-3 * sr[0]:
            assert abs(abs(U[:, i] @ Ur[:, i]) - 1.0) < 1e-9


def test_graded_matrix_relative_accuracy():
    rng = np.random.default_rng(11)
    Q1, _ = np.linalg.qr(rng.standard_normal((30, 10)))
    Q2, _ = np.linalg.qr(rng.standard_normal((10, 10)))
    sig = 10.0 ** -np.arange(10)
    A = (Q1 * sig) @ Q2.T
    U, s, V = svd(A)
    # normwise agreement with the exact values; graded values to high relative accuracy
    assert np.max(np.abs(s - sig)) <= 1e-14
    assert np.max(np.abs(s - sig) / sig) <= 1e-6


def test_two_by_two_closed_form():
    rng = np.random.default_rng(3)
    for _ in range(20):
        a, b, c, d = rng.standard_normal(4)
        A = np.array([[a, b], [c, d]])
        F = a * a + b * b + c * c + d * d
        D = abs(a * d - b * c)
        disc = np.sqrt(max(F * F - 4 * D * D, 0.0))
        s1 = np.sqrt((F + disc) / 2)
        s2 = D / s1
        _, s, _ = svd(A)
        assert abs(s[0] - s1) <= 1e-14 * s1 and abs(s[1] - s2) <= 1e-13 * s1


def test_special_cases():
    # diagonal with signs: sigma = sorted |d|; sign convention puts +1 in V
    A = np.diag([3.0, -5.0, 0.5, 2.0])
    U, s, V = svd(A)
    assert np.allclose(s, [5, 3, 2, 0.5], rtol=0, atol=1e-15)
    for j in range(4):
        i = np.argmax(np.abs(V[:, j]))
        assert V[i, j] > 0
    # zero matrix
    U, s, V = svd(np.zeros((6, 3)))
    assert np.all(s == 0.0)
    # rank deficient
    rng = np.random.default_rng(5)
    B = rng.standard_normal((20, 3)) @ rng.standard_normal((3, 8))
    U, s, V = svd(B)
    assert s[3] <= 1e-13 * s[0] and s[2] > 1e-3 * s[0]
    _check_factorisation(B, U, s, V)
    # repeated singular values (orthogonal matrix)
    Q, _ = np.linalg.qr(rng.standard_normal((9, 9)))
    U, s, V = svd(Q)
    assert np.max(np.abs(s - 1.0)) < 1e-14
    _check_factorisation(Q, U, s, V)


def test_eckart_young_truncation():
    rng = np.random.default_rng(8)
    A = rng.standard_normal((60, 25))
    s_all = svd(A)[1]
    for k in (1, 5, 24, 25):
        U, s, V = truncated_svd(A, k)
        err2 = np.linalg.norm(A - (U * s) @ V.T) ** 2
        assert abs(err2 - np.sum(s_all[k:] ** 2)) <= 1e-12 * np.sum(s_all ** 2)


def test_truncated_svd_keeps_the_numerical_rank():
    """Reading of TruncatedSVD(A, k) (Sec. 2.4.1) at FP64 rounding: singular
    values at or below RANK_TOL sigma_1 are zero, so k above the numerical
    rank keeps the numerical rank.  Spectra built from orthogonal factors put
    values on both sides of the cut; a product of rank 5 keeps 5 at any k."""
    from oracle.svd import RANK_TOL
    rng = np.random.default_rng(21)
    Q1, _ = np.linalg.qr(rng.standard_normal((30, 6)))
    Q2, _ = np.linalg.qr(rng.standard_normal((20, 6)))
    s_true = np.array([2.0, 1.0, 0.5, 2.0 * 50 * RANK_TOL, 2.0 * 0.02 * RANK_TOL, 0.0])
    A = (Q1 * s_true) @ Q2.T
    for k in (3, 4, 5, 6):
        U, s, V = truncated_svd(A, k)
        assert len(s) == min(k, 4), (k, s)
        assert np.max(np.abs(s - s_true[:len(s)])) <= 1e-14
    B = rng.standard_normal((50, 5)) @ rng.standard_normal((5, 40))
    for k in (5, 8, 12):
        U, s, V = truncated_svd(B, k)
        assert len(s) == 5
        assert np.linalg.norm(B - (U * s) @ V.T) <= 1e-13 * np.linalg.norm(B)
    assert truncated_svd(np.zeros((4, 3)), 2)[1].size == 0
