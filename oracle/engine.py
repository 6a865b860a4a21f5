"""Oracle stream driver: the engine loop of Algorithm 1, in FP64 on the CPU.

init: (U, Sigma, V) = TruncatedSVD(A_0, k), A = A_0, N_0 = ||A_0||_F^2 and
U_ref = U.  Per event (tick t = 1, 2, ...): append / modify A, run the
matching Brand update (row, column via transpose, or rank-1), truncate, then
evaluate the policy and refresh (TruncatedSVD(A_t, k_t)) if it fires; a
refresh stores U_ref = U (the reference for later angle measurements).

``force_refresh`` on ``step`` replaces the policy decision: parity tests log
the oracle's decisions and replay them, because a refresh fired one tick
apart turns rounding-level differences into drift-level ones.
"""
import numpy as np

from synth.factor_model import ROW, COL, ENTRY
from . import brand, metrics
from .policies import Policy, NONE, PERIODIC, ERROR, ANGLE, ADAPTIVE, DRIFT
from .svd import truncated_svd, singular_values


class OracleEngine:
    def __init__(self, A0, k, tol_rel=1e-10, policy=None, cgs2=False, drift=False):
        self.A = np.array(A0, dtype=np.float64, copy=True)
        self.k = int(k)
        self.policy = policy or Policy()
        self.k_max = self.policy.k_max or self.k
        self.tol_rel = tol_rel
        self.cgs2 = cgs2
        self.U, self.s, self.V = truncated_svd(self.A, self.k)
        self.N = float(np.sum(self.A * self.A))
        self.t = 0
        self.t_last = 0
        self.n_refresh = 0
        self.U_ref = self.U.copy()
        self.grow_pending = False
        self.last_novelty = float("nan")
        self.refresh_ticks = []
        self._init_drift(drift)

    def _init_drift(self, drift):
        # drift signals of the last update (Sections 3.2-3.3), formed when asked
        # for or when the policy adds them up
        self.drift = bool(drift) or self.policy.kind == DRIFT
        self.drift_acc = 0.0
        self.last_step_angle_U = self.last_step_angle_V = float("nan")
        self.last_spectrum_change = float("nan")

    @classmethod
    def from_state(cls, A, U, s, V, tol_rel=1e-10, policy=None, cgs2=False, drift=False):
        """Start from a given state (A_t, U, Sigma, V) instead of TruncatedSVD(A_0, k)."""
        eng = cls.__new__(cls)
        eng.A = np.array(A, dtype=np.float64, copy=True)
        eng.k = len(s)
        eng.policy = policy or Policy()
        eng.k_max = eng.policy.k_max or eng.k
        eng.tol_rel = tol_rel
        eng.cgs2 = cgs2
        eng.U, eng.s, eng.V = np.array(U, dtype=np.float64), np.array(s, dtype=np.float64), np.array(V, dtype=np.float64)
        eng.N = float(np.sum(eng.A * eng.A))
        eng.t = 0
        eng.t_last = 0
        eng.n_refresh = 0
        eng.U_ref = eng.U.copy()
        eng.grow_pending = False
        eng.last_novelty = float("nan")
        eng.refresh_ticks = []
        eng._init_drift(drift)
        return eng

    # ----------------------------------------------------------------- state
    @property
    def shape(self):
        return self.A.shape

    def refresh(self, store_reference=True):
        self.U, self.s, self.V = truncated_svd(self.A, self.k)
        if store_reference:
            self.U_ref = self.U.copy()
        self.t_last = self.t
        self.n_refresh += 1
        self.drift_acc = 0.0

    # ---------------------------------------------------------------- update
    def _k_keep(self):
        if self.grow_pending and self.k < self.k_max:
            return self.k + 1
        return self.k

    def apply(self, ev):
        """One Brand update (no policy)."""
        self.t += 1
        novelty = float("nan")
        U0, s0, V0 = self.U, self.s, self.V
        if ev.kind == ROW:
            x = np.asarray(ev.vec, dtype=np.float64)
            self.A = np.vstack([self.A, x[None, :]])
            self.N = metrics.fro2_row(self.N, x)
            self.U, self.s, self.V, info = brand.row_append(
                self.U, self.s, self.V, x, self._k_keep(), self.tol_rel, self.cgs2)
            novelty = info.rho / info.xnorm if info.xnorm > 0 else 0.0
        elif ev.kind == COL:
            y = np.asarray(ev.vec, dtype=np.float64)
            self.A = np.hstack([self.A, y[:, None]])
            self.N = metrics.fro2_col(self.N, y)
            self.U, self.s, self.V, info = brand.col_append(
                self.U, self.s, self.V, y, self._k_keep(), self.tol_rel, self.cgs2)
            novelty = info.rho / info.xnorm if info.xnorm > 0 else 0.0
        elif ev.kind == ENTRY:
            a_ij = float(self.A[ev.i, ev.j])
            self.A[ev.i, ev.j] += ev.delta
            self.N = metrics.fro2_entry(self.N, a_ij, ev.delta)
            self.U, self.s, self.V = brand.rank_one(self.U, self.s, self.V, ev.i, ev.j, ev.delta)
        else:
            raise ValueError("unknown event kind %r" % (ev.kind,))
        if len(self.s) > self.k:
            self.k = len(self.s)
            self.grow_pending = False
        self.last_novelty = novelty
        if self.drift:
            # largest principal angles between the previous spans (zero-padded
            # to the new rows) and the new ones; the spectrum's relative change
            self.last_step_angle_U = metrics.theta_max(U0, self.U)
            self.last_step_angle_V = metrics.theta_max(V0, self.V)
            self.last_spectrum_change = metrics.spectrum_change(s0, self.s)

    def decide(self, ev_kind):
        """Evaluate the policy after the update at tick t; may change k."""
        p = self.policy
        t = self.t
        if p.kind == NONE:
            return False
        if p.kind == PERIODIC:
            return p.period > 0 and t % p.period == 0
        if p.kind == ERROR:
            if p.check_every <= 0 or t % p.check_every != 0 or t - self.t_last < p.t_min:
                return False
            ratio = self.exact_metrics()["frob_ratio"]
            return bool(ratio > p.gamma)
        if p.kind == ANGLE:
            if t - self.t_last < max(p.t_min, 1):
                return False
            return bool(self.angle_ref(p.angle_scope) > p.theta_max)
        if p.kind == DRIFT:
            if np.isfinite(self.last_step_angle_U):
                self.drift_acc += self.last_step_angle_U
            return t - self.t_last >= max(p.t_min, 1) and self.drift_acc > p.theta_max
        if p.kind == ADAPTIVE:
            s2 = float(np.dot(self.s, self.s))
            low = s2 / self.N < p.tau - p.band
            novel = ev_kind in (ROW, COL) and self.last_novelty > p.eta
            if low or novel:
                if self.k < self.k_max:
                    self.grow_pending = True
            elif len(self.s) > p.k_min and (s2 - self.s[-1] ** 2) / self.N >= p.tau + p.band:
                self.U, self.s, self.V = self.U[:, :-1], self.s[:-1], self.V[:, :-1]
                self.k = len(self.s)
                self.grow_pending = False
            return p.period > 0 and t % p.period == 0
        raise ValueError("unknown policy kind")

    def step(self, ev, force_refresh=None):
        """Algorithm 1 body: update, truncate, policy, optional refresh.

        Returns True if a refresh ran after this update."""
        self.apply(ev)
        fire = self.decide(ev.kind) if force_refresh is None else bool(force_refresh)
        if fire:
            self.refresh(store_reference=True)
            self.refresh_ticks.append(self.t)
        return fire

    # --------------------------------------------------------------- metrics
    def angle_ref(self, scope=0):
        j = scope if scope > 0 else metrics.gap_separated_scope(self.s)
        j = min(j, self.U.shape[1], self.U_ref.shape[1])
        return metrics.theta_ref(self.U_ref[:, :j], self.U[:, :j])

    def cheap_metrics(self):
        s2 = float(np.dot(self.s, self.s))
        m, n = self.A.shape
        return {"t": self.t, "m": m, "n": n, "k": len(self.s), "fro2_A": self.N,
                "sigma2_sum": s2, "evr": metrics.evr(self.s, self.N),
                "novelty": self.last_novelty, "n_refresh": self.n_refresh,
                "t_last_refresh": self.t_last}

    def exact_metrics(self, with_angles=False):
        out = self.cheap_metrics()
        sig = singular_values(self.A)
        e_inc, e_opt, gap, ratio = metrics.frob_errors(self.A, self.U, self.s, self.V, sig)
        out.update(frob_error=e_inc, frob_opt=e_opt, frob_gap=gap, frob_ratio=ratio,
                   fro2_direct=float(np.sum(self.A * self.A)))
        if with_angles:
            from .svd import svd
            Uf = svd(self.A)[0]
            k = len(self.s)
            out["angle_opt"] = metrics.theta_max(Uf[:, :k], self.U)
            out["angle_ref"] = self.angle_ref(0)
            out["ortho_U"] = metrics.orthogonality(self.U)
            out["ortho_V"] = metrics.orthogonality(self.V)
        return out
