"""Oracle readout of a returns stream (FP64), Section 5 -- TEST INFRASTRUCTURE.

* Causal de-meaning (Section 5.1): each column keeps its expanding mean by the
  recurrence mu_t = mu_{t-1} + (r_t - mu_{t-1}) / t, and the row appended at
  time t is R_t = r_t - mu_t (only returns up to and including t are used).
* Low-rank covariances (Section 5.3, eq. low-rank-covariances):
  Sigma_k = V_k diag(sigma_1^2 .. sigma_k^2) V_k^T / (t - 1), t the number of
  rows of the centred panel, from the incremental factors (Sigma_inc,k) or
  from the exact truncated SVD (Sigma_full,k).
* err_cov = ||Sigma_inc,k - Sigma_full,k||_F / ||Sigma_full,k||_F (eq. cov-error).
* Portfolio volatility sigma = sqrt(w^T Sigma_k w) (eq. portfolio-vol) and
  err_risk = |sigma_inc - sigma_full| / sigma_full (eq. risk-error).

Every function forms the n x n matrices densely, as the definitions read;
nothing is blocked or reordered.
"""
import numpy as np


def causal_center(r, mu=None, t0=0):
    """Centre the rows of r (rows x n) by the expanding-mean recurrence.

    mu: the mean after t0 earlier rows (ignored when t0 == 0).  Returns
    (centred rows, mean after the last row)."""
    r = np.asarray(r, dtype=np.float64)
    m = np.zeros(r.shape[1]) if t0 == 0 else np.array(mu, dtype=np.float64, copy=True)
    out = np.empty_like(r)
    for q in range(r.shape[0]):
        t = t0 + q + 1
        m = m + (r[q] - m) / t
        out[q] = r[q] - m
    return out, m


def low_rank_cov(V, s, t):
    """V_k diag(s^2) V_k^T / (t - 1) (n x n)."""
    V = np.asarray(V, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    return (V * (s * s)) @ V.T / (t - 1)


def cov_error(V_inc, s_inc, V_full, s_full, t):
    C_inc = low_rank_cov(V_inc, s_inc, t)
    C_full = low_rank_cov(V_full, s_full, t)
    return float(np.linalg.norm(C_inc - C_full) / np.linalg.norm(C_full))


def portfolio_vol(V, s, t, w):
    # Sigma_k is positive semidefinite: a negative w^T Sigma_k w is rounding
    w = np.asarray(w, dtype=np.float64)
    return float(np.sqrt(max(w @ low_rank_cov(V, s, t) @ w, 0.0)))


def risk_error(vol_inc, vol_full):
    return abs(vol_inc - vol_full) / vol_full
