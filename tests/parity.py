"""Comparison of a GPU state (U, S, V) with the oracle's, in FP64 on the host.

* reconstruction: ||A_g - A_o||_F / ||A_o||_F with A = U diag(S) V^T, formed
  without the m x n products: with thin QRs [U_g U_o] = Qu Ru and
  [V_g V_o] = Qv Rv, A_g - A_o = Qu (Ru_g S_g Rv_g^T - Ru_o S_o Rv_o^T) Qv^T.
* sigma: max_i |s_g,i - s_o,i| / s_o,1 (normwise; Weyl bounds it by the
  perturbation's norm).
* angle: largest principal angle (sine form) between the leading j columns,
  j = the oracle spectrum's gap-separated scope (and the full-k angle).
"""
import numpy as np


def recon_rel_err(Ug, Sg, Vg, Uo, So, Vo):
    kg, ko = len(Sg), len(So)
    m = max(Ug.shape[0], Uo.shape[0])
    n = max(Vg.shape[0], Vo.shape[0])

    def pad(Q, r):
        if Q.shape[0] == r:
            return Q
        out = np.zeros((r, Q.shape[1]))
        out[:Q.shape[0]] = Q
        return out

    Qu, Ru = np.linalg.qr(np.hstack([pad(Ug, m), pad(Uo, m)]))
    Qv, Rv = np.linalg.qr(np.hstack([pad(Vg, n), pad(Vo, n)]))
    D = (Ru[:, :kg] * Sg) @ Rv[:, :kg].T - (Ru[:, kg:] * So) @ Rv[:, kg:].T
    return float(np.linalg.norm(D) / np.linalg.norm(So))


def sigma_err(Sg, So):
    k = min(len(Sg), len(So))
    e = np.max(np.abs(Sg[:k] - So[:k])) / So[0]
    if len(Sg) != len(So):
        e = max(e, 1.0)
    return float(e)


def theta(Q1, Q2):
    """Largest principal angle between span(Q1), span(Q2) (same dims)."""
    Q1, _ = np.linalg.qr(Q1)
    Q2, _ = np.linalg.qr(Q2)
    C = Q1.T @ Q2
    c = np.linalg.svd(C, compute_uv=False)
    th = float(np.arccos(np.clip(c.min(), 0.0, 1.0)))
    if th < 0.1:
        th = float(np.arcsin(min(1.0, np.linalg.norm(Q2 - Q1 @ C, 2))))
    return th


def gap_scope(s, rel_gap=0.05):
    k = len(s)
    best, best_gap = k, -1.0
    for j in range(1, k):
        g = (s[j - 1] - s[j]) / s[j - 1] if s[j - 1] > 0 else 0.0
        if g > best_gap:
            best, best_gap = j, g
    return best if best_gap >= rel_gap else k


def compare(gpu, orc):
    """gpu, orc: (U, S, V) triples.  Returns a dict of errors."""
    Ug, Sg, Vg = gpu
    Uo, So, Vo = orc
    j = gap_scope(So)
    return {
        "recon": recon_rel_err(Ug, Sg, Vg, Uo, So, Vo),
        "sigma": sigma_err(Sg, So),
        "angle_scope": j,
        "angle_U": theta(Ug[:, :j], Uo[:, :j]),
        "angle_V": theta(Vg[:, :j], Vo[:, :j]),
        "angle_U_full": theta(Ug, Uo) if len(Sg) == len(So) else float("nan"),
        "ortho_U": float(np.max(np.abs(Ug.T @ Ug - np.eye(len(Sg))))),
        "ortho_V": float(np.max(np.abs(Vg.T @ Vg - np.eye(len(Sg))))),
    }
