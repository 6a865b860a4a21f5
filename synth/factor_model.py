"""Synthetic factor-model return streams (inputs only).

Model: every entry of the panel is A[i, j] = f_i . b_j + noise * eps_ij with
loadings b_j ~ N(0, I_K) per column, factors f_i ~ N(0, diag(lambda)) per row
and eps ~ N(0, 1).  Every quantity is regenerated from its own Philox
counter, so a row appended at row index i and a column appended at column
index j see exactly the factors / loadings the panel already used:

* b_j   = normals(purpose LOAD,  tick j)[:K]
* f_i   = sqrt(lambda) * normals(purpose FACT, tick i)[:K]
* noise of the entries created with row i    = normals(NOISE_ROW, tick i)
* noise of the entries created with column j = normals(NOISE_COL, tick j)

Each entry's noise is drawn once: by the row that created it (initial rows
and row appends) or by the column that created it (column appends).

Factor variances: lambda_j = 4 * 16^(-j/(K-1)), j = 0..K-1, which gives
(4, 2, 1, 0.5, 0.25) for K = 5 and extends the same geometric decay to the
20- and 40-factor panels.
"""
from dataclasses import dataclass
from typing import Optional

import numpy as np

from .philox import normals, uniforms

ROW, COL, ENTRY = 0, 1, 2

P_LOAD, P_FACT, P_NOISE_ROW, P_NOISE_COL, P_EVENT, P_DELTA, P_PERM = 1, 2, 3, 4, 5, 6, 7


def factor_lambdas(K):
    if K == 1:
        return np.array([4.0])
    j = np.arange(K, dtype=np.float64)
    return 4.0 * 16.0 ** (-j / (K - 1))


@dataclass
class Event:
    kind: int
    t: int
    vec: Optional[np.ndarray] = None   # row x (ROW) or column y (COL)
    i: int = -1
    j: int = -1
    delta: float = 0.0


class FactorStream:
    """One synthetic stream: loadings, factors and noise keyed by (seed, stream)."""

    def __init__(self, seed, stream, n0, K, noise=0.1, lambdas=None):
        self.seed = int(seed)
        self.stream = int(stream)
        self.n0 = int(n0)
        self.K = int(K)
        self.noise = float(noise)
        self.lam = np.asarray(lambdas if lambdas is not None else factor_lambdas(K), dtype=np.float64)

    def _nrm(self, purpose, ticks, count):
        return normals(self.seed, self.stream, purpose, ticks, count)

    def loadings(self, j0, j1):
        return self._nrm(P_LOAD, np.arange(j0, j1), self.K)

    def factors(self, i0, i1):
        return self._nrm(P_FACT, np.arange(i0, i1), self.K) * np.sqrt(self.lam)[None, :]

    @staticmethod
    def _outer_sum(F, B):
        # sum_l F[:, l] B[:, l]^T in a fixed order (l = 0..K-1, no fused ops),
        # the order the device generator uses as well
        out = np.zeros((F.shape[0], B.shape[0]))
        for l in range(F.shape[1]):
            out += F[:, l:l + 1] * B[None, :, l]
        return out

    def initial(self, m0):
        F = self.factors(0, m0)
        B = self.loadings(0, self.n0)
        return self._outer_sum(F, B) + self.noise * self._nrm(P_NOISE_ROW, np.arange(m0), self.n0)

    def row(self, i, n_cols):
        F = self.factors(i, i + 1)
        B = self.loadings(0, n_cols)
        return (self._outer_sum(F, B) + self.noise * self._nrm(P_NOISE_ROW, [i], n_cols))[0]

    def col(self, j, m_rows):
        F = self.factors(0, m_rows)
        B = self.loadings(j, j + 1)
        return (self._outer_sum(F, B) + self.noise * self._nrm(P_NOISE_COL, [j], m_rows).T)[:, 0]

    def entry_params(self, t, m_t, n_t, delta_std=0.5):
        u = uniforms(self.seed, self.stream, P_EVENT, [t], 4)[0]
        i = min(int(np.floor(u[2] * m_t)), m_t - 1)
        j = min(int(np.floor(u[3] * n_t)), n_t - 1)
        d = delta_std * self._nrm(P_DELTA, [t], 1)[0, 0]
        return i, j, float(d)

    def materialize(self, kinds, m0, t0=1, delta_std=0.5):
        """Turn a list of event kinds into concrete events (payloads drawn now).

        Tick numbering starts at t0 (the first update is t = 1, as in the
        engine loop); shapes grow as rows and columns are appended."""
        m, n = int(m0), int(self.n0)
        out = []
        for off, kind in enumerate(kinds):
            t = t0 + off
            if kind == ROW:
                out.append(Event(ROW, t, vec=self.row(m, n)))
                m += 1
            elif kind == COL:
                out.append(Event(COL, t, vec=self.col(n, m)))
                n += 1
            else:
                i, j, d = self.entry_params(t, m, n, delta_std)
                out.append(Event(ENTRY, t, i=i, j=j, delta=d))
        return out


def event_schedule_c0(seed, stream, n_rows=1000, n_entries=200):
    """Row appends and entry updates in a seeded random interleaving."""
    total = n_rows + n_entries
    u = uniforms(seed, stream, P_PERM, [0], total)[0]
    kinds = np.full(total, ROW, dtype=np.int64)
    kinds[np.argsort(u, kind="stable")[:n_entries]] = ENTRY
    return kinds.tolist()


def event_schedule_iid(seed, stream, T, mix=(0.8, 0.1, 0.1), t0=1):
    """Event kinds drawn i.i.d. from the categorical (row, col, entry) mix."""
    u = uniforms(seed, stream, P_EVENT, np.arange(t0, t0 + T), 2)[:, 0]
    c1 = mix[0]
    c2 = mix[0] + mix[1]
    kinds = np.where(u < c1, ROW, np.where(u < c2, COL, ENTRY))
    return kinds.astype(np.int64).tolist()
