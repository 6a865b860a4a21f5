"""Oracle refresh and rank policies (Section 3), evaluated after each update.

* Periodic (eq. periodic-refresh-rule): refresh after the update at tick t
  iff t = 0 mod T; t counts every update and is not reset by a refresh.
* Error threshold (eq. error-refresh-rule): at check ticks (t = 0 mod
  check_every) refresh iff frob_ratio(t) > gamma and t - t_last >= t_min.
  The oracle evaluates frob_ratio exactly from a full SVD of A_t.
* Angle threshold (Section 3.3): refresh iff the largest principal angle
  theta_ref between the reference subspace stored at the last refresh and
  the current one (on the reference's rows) exceeds theta_max, measured on
  the leading ``scope`` columns.  The default scope is the leading
  gap-separated subspace of the maintained spectrum (the largest relative
  gap, if >= 5%); beyond it the truncation cuts through a cluster of nearly
  equal singular values whose directions are not determined to rounding.
  The paper's own trigger, angle_to_opt, needs a full SVD per tick; theta_ref
  is the cheap drift signal the same section lists as its practical stand-in.
* Adaptive rank (eqs. evr-rank-rule, novelty-rank-rule, Section 3.4): with
  target tau and band b, schedule growth by one (the next append keeps one
  more Brand triplet) when EVR < tau - b or the append just made had
  ||z|| > eta ||x||; on ticks with neither signal, shrink by one (drop the
  last triplet at once) when the model without its last triplet still
  explains >= tau + b.  Rank stays in [k_min, k_max]; a periodic refresh
  every ``period`` ticks runs at the current rank.
* Drift surrogate (Sections 3.2-3.3; the paper names the angle between
  successive subspaces as a cheap trigger but gives no rule): add up the
  step angle of U (the largest principal angle between span(U_{t-1}),
  zero-padded to the new rows, and span(U_t)) after every update and
  refresh iff the sum since the last refresh exceeds theta_max and
  t - t_last >= t_min.  The largest principal angle is a metric on subspaces
  of one dimension, so while the rank holds the sum bounds the angle between
  the span at the last refresh and the current one; no A is read.
"""
from dataclasses import dataclass

NONE, PERIODIC, ERROR, ANGLE, ADAPTIVE, DRIFT = 0, 1, 2, 3, 4, 5


@dataclass
class Policy:
    kind: int = NONE
    period: int = 0
    gamma: float = 1.05
    check_every: int = 100
    t_min: int = 0
    theta_max: float = 1e-3
    angle_scope: int = 0          # 0 = leading gap-separated subspace
    tau: float = 0.95
    band: float = 0.01
    eta: float = 0.5
    k_min: int = 1
    k_max: int = 0                # 0 = the initial k

    @staticmethod
    def periodic(T):
        return Policy(kind=PERIODIC, period=int(T))

    @staticmethod
    def error(gamma=1.05, check_every=100, t_min=None):
        return Policy(kind=ERROR, gamma=gamma, check_every=check_every,
                      t_min=check_every if t_min is None else t_min)

    @staticmethod
    def angle(theta_max=1e-3, scope=0, t_min=1):
        return Policy(kind=ANGLE, theta_max=theta_max, angle_scope=scope, t_min=t_min)

    @staticmethod
    def drift(theta_max=1e-2, t_min=1):
        return Policy(kind=DRIFT, theta_max=theta_max, t_min=t_min)

    @staticmethod
    def adaptive(tau=0.95, band=0.01, eta=0.5, k_min=1, k_max=0, period=500):
        return Policy(kind=ADAPTIVE, tau=tau, band=band, eta=eta, k_min=k_min, k_max=k_max, period=period)
