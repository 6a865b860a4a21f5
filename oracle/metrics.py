"""Oracle metrics (FP64): Section 2.4.2 (principal angles) and Section 2.5.

* E_inc = ||A - U Sigma V^T||_F and E_opt = ||A - A_k*||_F (eq. frob-errors);
  frob_gap = E_inc - E_opt and frob_ratio = E_inc / E_opt (eq. frob-ratio),
  NaN when E_opt is numerically zero.
* EVR = ||Sigma||_F^2 / N_t (eq. evr) with N_t = ||A_t||_F^2 tracked by the
  recurrences of Section 2.5.2.
* theta_max(Q1, Q2) = arccos sigma_min(Q1^T Q2) (eq. theta-max).  Near zero
  the cosine loses digits, so angles below 0.1 rad use the sine form
  sin theta_max = ||Q2 - Q1 (Q1^T Q2)||_2 (Bjorck and Golub), valid when
  dim span(Q2) <= dim span(Q1).  A basis with fewer rows is padded with zero
  rows (rows appended after it was taken).
* theta_ref (eq. angle-metrics-ref) compares U_ref with U_t restricted to the
  rows U_ref has (re-orthonormalised).  Rows appended since the reference add
  weight of about sqrt(rows added / rows) outside the zero-padded reference
  however little the subspace turned, so the padded angle measures growth,
  not drift; on the reference rows it measures drift alone.
* drift signals that need no A (the surrogates of Sections 3.2-3.3): the
  step angles theta_max(U_{t-1}, U_t), theta_max(V_{t-1}, V_t) of one
  update, and spectrum_change = ||sigma_t - sigma_{t-1}|| / ||sigma_{t-1}||.
* the default angle scope is the leading gap-separated subspace: the j < k
  with the largest relative gap (s_j - s_{j+1}) / s_j, if that gap is at
  least 5%, else all k columns.
"""
import numpy as np

from .svd import svd


def fro2_row(N, x):
    return N + float(np.dot(x, x))


def fro2_col(N, y):
    return N + float(np.dot(y, y))


def fro2_entry(N, a_ij, delta):
    return N + 2.0 * delta * a_ij + delta * delta


def evr(s, N):
    return float(np.dot(s, s)) / N if N > 0 else float("nan")


def frob_errors(A, U, s, V, sigma_full):
    """(E_inc, E_opt, gap, ratio) for the maintained rank-k model."""
    k = len(s)
    E_inc = float(np.linalg.norm(A - (U * s[None, :]) @ V.T))
    tail = sigma_full[k:]
    E_opt = float(np.sqrt(np.dot(tail, tail)))
    normA = float(np.linalg.norm(A))
    ratio = E_inc / E_opt if E_opt > 1e-14 * normA else float("nan")
    return E_inc, E_opt, E_inc - E_opt, ratio


def _pad_rows(Q, m):
    if Q.shape[0] == m:
        return Q
    out = np.zeros((m, Q.shape[1]))
    out[:Q.shape[0]] = Q
    return out


def principal_cosines(Q1, Q2):
    m = max(Q1.shape[0], Q2.shape[0])
    Q1 = _pad_rows(Q1, m)
    Q2 = _pad_rows(Q2, m)
    return np.clip(svd(Q1.T @ Q2)[1], 0.0, 1.0)


def theta_max(Q1, Q2):
    """Largest principal angle between span(Q1) and span(Q2), radians."""
    m = max(Q1.shape[0], Q2.shape[0])
    Q1 = _pad_rows(Q1, m)
    Q2 = _pad_rows(Q2, m)
    if Q2.shape[1] > Q1.shape[1]:
        Q1, Q2 = Q2, Q1
    C = Q1.T @ Q2
    cmin = float(np.clip(svd(C)[1].min(), 0.0, 1.0))
    theta = float(np.arccos(cmin))
    if theta < 0.1:
        R = Q2 - Q1 @ C
        smax = float(svd(R)[1].max()) if R.size else 0.0
        theta = float(np.arcsin(min(smax, 1.0)))
    return theta


def spectrum_change(s_prev, s_new):
    """||sigma_t - sigma_{t-1}||_2 / ||sigma_{t-1}||_2, the shorter vector
    zero-padded: the spectrum-change surrogate of the error-based refresh
    (Section 3.2).  NaN when sigma_{t-1} is zero."""
    n = max(len(s_prev), len(s_new))
    a = np.zeros(n)
    b = np.zeros(n)
    a[:len(s_prev)] = s_prev
    b[:len(s_new)] = s_new
    den = float(np.linalg.norm(a))
    return float(np.linalg.norm(b - a)) / den if den > 0.0 else float("nan")


def theta_ref(U_ref, U_t):
    """Largest angle between span(U_ref) and span(U_t restricted to U_ref's rows)."""
    m_ref = U_ref.shape[0]
    W = U_t[:m_ref, :]
    Q = svd(W)[0][:, :W.shape[1]] if W.shape[0] >= W.shape[1] else svd(W)[0]
    return theta_max(U_ref, Q)


def orthogonality(Q):
    """||Q^T Q - I||_2."""
    E = Q.T @ Q - np.eye(Q.shape[1])
    return float(svd(E)[1].max()) if E.size else 0.0


def gap_separated_scope(s, rel_gap=0.05):
    """The j < k (1-based) maximising (s_j - s_{j+1}) / s_j if that gap is at
    least rel_gap (first such j on ties), else k."""
    k = len(s)
    best, best_gap = k, -1.0
    for j in range(1, k):
        g = (s[j - 1] - s[j]) / s[j - 1] if s[j - 1] > 0 else 0.0
        if g > best_gap:
            best, best_gap = j, g
    return best if best_gap >= rel_gap else k
