"""Pins of the oracle's finance readout (Section 5) against closed forms.

* causal de-meaning: the recurrence's mean equals the expanding mean formed
  as cumulative sums over 1..t; the first centred row is zero; a constant
  column centres to zero; splitting the rows across calls changes nothing.
* low-rank covariance with k = rank equals the sample covariance
  R^T R / (t - 1) (eq. sample-covariance), factors from LAPACK's SVD.
* covariance error: scaling every sigma by a gives |a^2 - 1|; orthogonal
  subspaces give sqrt(sum s_inc^4 + sum s_full^4) / sqrt(sum s_full^4).
* portfolio volatility: w = e_j reads the covariance's diagonal; w along a
  right singular vector v_i gives sigma_i / sqrt(t - 1); w orthogonal to the
  subspace gives 0.
"""
import numpy as np
import pytest

from oracle import finance as F


def _returns(rng, t, n):
    return 0.01 * rng.standard_normal((t, n)) + 0.002 * rng.standard_normal(n)


def test_causal_center_is_the_expanding_mean():
    rng = np.random.default_rng(0)
    r = _returns(rng, 200, 17)
    out, mu = F.causal_center(r)
    expanding = np.cumsum(r, axis=0) / np.arange(1, 201)[:, None]
    assert np.allclose(out, r - expanding, rtol=0, atol=1e-15)
    assert np.allclose(mu, r.mean(axis=0), rtol=0, atol=1e-16)
    assert np.array_equal(out[0], np.zeros(17))


def test_causal_center_constant_column_and_split_calls():
    rng = np.random.default_rng(1)
    r = _returns(rng, 90, 6)
    r[:, 2] = 0.75
    out, mu = F.causal_center(r)
    assert np.array_equal(out[:, 2], np.zeros(90))
    a, mu_a = F.causal_center(r[:37])
    b, mu_b = F.causal_center(r[37:], mu_a, 37)
    assert np.array_equal(np.vstack([a, b]), out)
    assert np.array_equal(mu_b, mu)


def test_full_rank_covariance_is_the_sample_covariance():
    rng = np.random.default_rng(2)
    R, _ = F.causal_center(_returns(rng, 120, 15))
    _, s, Vt = np.linalg.svd(R, full_matrices=False)
    C = F.low_rank_cov(Vt.T, s, 120)
    S = R.T @ R / 119
    assert np.abs(C - S).max() <= 1e-12 * np.abs(S).max()


def test_cov_error_closed_forms():
    rng = np.random.default_rng(3)
    V, _ = np.linalg.qr(rng.standard_normal((40, 5)))
    s = np.array([5.0, 3.0, 2.0, 1.0, 0.5])
    assert F.cov_error(V, s, V, s, 100) == 0.0
    for a in (0.9, 1.1, 2.0):
        assert abs(F.cov_error(V, a * s, V, s, 100) - abs(a * a - 1)) <= 1e-13
    Q, _ = np.linalg.qr(rng.standard_normal((40, 10)))
    V1, V2 = Q[:, :5], Q[:, 5:]
    s2 = np.array([4.0, 2.5, 1.5, 0.7, 0.2])
    want = np.sqrt(np.sum(s ** 4) + np.sum(s2 ** 4)) / np.sqrt(np.sum(s2 ** 4))
    assert abs(F.cov_error(V1, s, V2, s2, 100) - want) <= 1e-12 * want


def test_portfolio_vol_closed_forms():
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((30, 6)))
    V = Q[:, :5]
    s = np.array([6.0, 4.0, 2.0, 1.0, 0.3])
    t = 250
    C = F.low_rank_cov(V, s, t)
    for j in (0, 7, 29):
        e = np.zeros(30)
        e[j] = 1.0
        direct = np.sqrt(np.sum(s * s * V[j] ** 2) / (t - 1))
        assert abs(F.portfolio_vol(V, s, t, e) - direct) <= 1e-15 + 1e-13 * direct
        assert abs(F.portfolio_vol(V, s, t, e) ** 2 - C[j, j]) <= 1e-13 * C[j, j]
    for i in range(5):
        assert abs(F.portfolio_vol(V, s, t, V[:, i]) - s[i] / np.sqrt(t - 1)) <= 1e-13 * s[i]
    assert F.portfolio_vol(V, s, t, Q[:, 5]) <= 1e-14
    assert F.risk_error(1.1, 1.0) == pytest.approx(0.1, abs=1e-15)
