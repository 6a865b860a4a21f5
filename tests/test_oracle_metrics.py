"""Pins of the oracle's metrics: N_t recurrences, Eckart-Young, angles, EVR, ratio."""
import numpy as np
import pytest
import scipy.linalg

from oracle import metrics
from oracle.svd import svd, truncated_svd


def test_fro2_recurrences_match_direct_sum():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((10, 6))
    N = float(np.sum(A * A))
    for step in range(30):
        kind = step % 3
        if kind == 0:
            x = rng.standard_normal(A.shape[1])
            N = metrics.fro2_row(N, x)
            A = np.vstack([A, x])
        elif kind == 1:
            y = rng.standard_normal(A.shape[0])
            N = metrics.fro2_col(N, y)
            A = np.hstack([A, y[:, None]])
        else:
            i, j, d = rng.integers(A.shape[0]), rng.integers(A.shape[1]), rng.standard_normal()
            N = metrics.fro2_entry(N, A[i, j], d)
            A[i, j] += d
    assert abs(N - np.sum(A * A)) <= 1e-12 * N


@pytest.mark.parametrize("a", [1e-10, 1e-6, 1e-3, 0.3, 1.2, np.pi / 2])
def test_theta_closed_form_two_lines(a):
    e1 = np.array([[1.0], [0.0], [0.0]])
    q = np.array([[np.cos(a)], [np.sin(a)], [0.0]])
    th = metrics.theta_max(e1, q)
    assert abs(th - a) <= 1e-14 + 1e-12 * a


def test_theta_invariant_and_against_scipy():
    rng = np.random.default_rng(1)
    Q1, _ = np.linalg.qr(rng.standard_normal((50, 6)))
    R = rng.standard_normal((6, 6)) + 3 * np.eye(6)
    Q2, _ = np.linalg.qr(Q1 @ R)
    assert metrics.theta_max(Q1, Q2) < 1e-14
    Q3, _ = np.linalg.qr(Q1 + 0.05 * rng.standard_normal((50, 6)))
    ref = np.max(scipy.linalg.subspace_angles(Q1, Q3))
    assert abs(metrics.theta_max(Q1, Q3) - ref) < 1e-12
    Q4, _ = np.linalg.qr(rng.standard_normal((50, 6)))
    ref = np.max(scipy.linalg.subspace_angles(Q1, Q4))
    assert abs(metrics.theta_max(Q1, Q4) - ref) < 1e-10
    c = metrics.principal_cosines(Q1, Q4)
    assert np.all((c >= 0) & (c <= 1))


def test_theta_pads_rows_of_older_basis():
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((20, 3)))
    Qlong = np.vstack([Q, np.zeros((5, 3))])
    assert metrics.theta_max(Q, Qlong) < 1e-14


def test_frob_errors_eckart_young_and_ratio():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 30))
    sig = svd(A)[1]
    U, s, V = truncated_svd(A, 8)
    e_inc, e_opt, gap, ratio = metrics.frob_errors(A, U, s, V, sig)
    assert abs(e_inc - e_opt) <= 1e-12 * e_opt and abs(ratio - 1.0) < 1e-12
    # any other rank-8 model is worse: ratio >= 1 (Eckart-Young corollary)
    Q, _ = np.linalg.qr(U + 0.1 * rng.standard_normal(U.shape))
    e_inc2, _, gap2, ratio2 = metrics.frob_errors(A, Q, s, V, sig)
    assert ratio2 > 1.0 and gap2 > 0
    assert 0.0 < metrics.evr(s, np.sum(A * A)) <= 1.0
    # zero optimal error -> ratio undefined
    B = rng.standard_normal((10, 2)) @ rng.standard_normal((2, 8))
    U, s, V = truncated_svd(B, 3)
    _, e_opt, _, ratio = metrics.frob_errors(B, U, s, V, svd(B)[1])
    assert np.isnan(ratio)


def test_gap_scope():
    assert metrics.gap_separated_scope(np.array([10.0, 9.9, 5.0, 4.99, 4.98])) == 2
    assert metrics.gap_separated_scope(np.array([10.0, 9.99, 9.98])) == 3
    assert metrics.gap_separated_scope(np.array([300.0, 200, 100, 3.0, 2.9, 2.8])) == 3


def test_theta_ref_ignores_row_growth_but_sees_rotation():
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((30, 4)))
    # same subspace on the old rows, plus new rows: zero restricted angle
    grown = np.vstack([Q, 0.3 * rng.standard_normal((6, 4))])
    grown, _ = np.linalg.qr(grown)
    assert metrics.theta_max(Q, grown) > 0.1
    assert metrics.theta_ref(Q, grown) < 1e-13
    # a genuine rotation by angle a inside the old rows is seen
    a = 1e-4
    P = np.vstack([Q[:, :3].T, np.cos(a) * Q[:, 3] + np.sin(a) * np.linalg.qr(
        np.column_stack([Q, rng.standard_normal(30)]))[0][:, 4]]).T
    assert abs(metrics.theta_ref(Q, P) - a) < 1e-12


def test_orthogonality_known_answer():
    """||Q^T Q - I||_2 for Q = O diag(d) P^T (O with orthonormal columns, P
    orthogonal) is max_i |d_i^2 - 1|: the spectral norm, not the Frobenius
    norm (0.2315 here) nor the largest entry of the rotated Gram residual."""
    from oracle.metrics import orthogonality
    rng = np.random.default_rng(5)
    d = np.array([1.1, 0.95, 1.0, 1.0 + 1e-9])
    O, _ = np.linalg.qr(rng.standard_normal((30, 4)))
    P, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    Q = O @ np.diag(d) @ P.T
    assert abs(orthogonality(Q) - 0.21) <= 1e-14
    E = Q.T @ Q - np.eye(4)
    assert abs(np.linalg.norm(E) - 0.21) > 1e-2          # Frobenius differs
    assert np.max(np.abs(E)) < 0.21 - 1e-3               # so does the largest entry
    # an exactly orthonormal basis has zero residual; a scaled one |c^2 - 1|
    assert orthogonality(O) <= 1e-15
    assert abs(orthogonality(1.5 * O) - 1.25) <= 1e-14
