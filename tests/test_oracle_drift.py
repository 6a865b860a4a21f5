"""Pins of the oracle's drift signals (the surrogates of Sections 3.2-3.3)
against closed forms and explicit matrices, independent of the engine loop.

* 1 x 2 closed form, k = 1: A_0 = [1 0]; appending [0 a] with a > 1 turns
  both spans by pi / 2 and changes the spectrum by |a - 1|; with a < 1 nothing
  turns and the spectrum is unchanged.
* k = n (full column rank), row append: V spans R^n before and after (angle
  0); U's step angle equals the largest principal angle between
  range([A_0; 0]) and range(A_1), from QR factors of the explicit matrices
  and the sine form ||(I - Q_0 Q_0^T) Q_1||_2; the spectrum change equals
  the one of LAPACK's singular values of A_0 and A_1.
* k = m (full row rank), column append: the mirror image (U's angle 0).
* square full rank, entry update: both spans are R^n (angles 0) and the
  spectrum change is LAPACK's.
A swapped U / V, padding at the wrong end or the wrong normaliser fails one
of them.
"""
import numpy as np

from oracle.engine import OracleEngine
from synth import ROW, COL, ENTRY


class _Ev:
    def __init__(self, kind, vec=None, i=0, j=0, delta=0.0):
        self.kind, self.vec, self.i, self.j, self.delta = kind, vec, i, j, delta


def _angle(A0_pad, A1):
    Q0, _ = np.linalg.qr(A0_pad)
    Q1, _ = np.linalg.qr(A1)
    R = Q1 - Q0 @ (Q0.T @ Q1)
    return float(np.arcsin(min(1.0, np.linalg.svd(R, compute_uv=False).max())))


def _spec(A0, A1):
    s0 = np.linalg.svd(A0, compute_uv=False)
    s1 = np.linalg.svd(A1, compute_uv=False)
    n = max(len(s0), len(s1))
    a, b = np.zeros(n), np.zeros(n)
    a[:len(s0)], b[:len(s1)] = s0, s1
    return float(np.linalg.norm(b - a) / np.linalg.norm(a))


def test_one_by_two_closed_form():
    o = OracleEngine(np.array([[1.0, 0.0]]), 1, drift=True)
    o.apply(_Ev(ROW, np.array([0.0, 2.0])))
    assert abs(o.last_step_angle_U - np.pi / 2) <= 1e-12
    assert abs(o.last_step_angle_V - np.pi / 2) <= 1e-12
    assert abs(o.last_spectrum_change - 1.0) <= 1e-14
    o = OracleEngine(np.array([[1.0, 0.0]]), 1, drift=True)
    o.apply(_Ev(ROW, np.array([0.0, 0.5])))
    assert o.last_step_angle_U <= 1e-14 and o.last_step_angle_V <= 1e-14
    assert o.last_spectrum_change <= 1e-14


def test_row_append_full_column_rank():
    rng = np.random.default_rng(0)
    A0 = rng.standard_normal((30, 6))
    o = OracleEngine(A0, 6, drift=True)
    A = A0
    for q in range(4):
        x = rng.standard_normal(6) * (1 + q)
        o.apply(_Ev(ROW, x))
        A1 = np.vstack([A, x[None, :]])
        assert o.last_step_angle_V <= 1e-12
        want = _angle(np.vstack([A, np.zeros((1, 6))]), A1)
        assert want > 0.05
        assert abs(o.last_step_angle_U - want) <= 1e-12
        assert abs(o.last_spectrum_change - _spec(A, A1)) <= 1e-13
        A = A1


def test_col_append_full_row_rank():
    rng = np.random.default_rng(1)
    A0 = rng.standard_normal((6, 30))
    o = OracleEngine(A0, 6, drift=True)
    y = rng.standard_normal(6)
    o.apply(_Ev(COL, y))
    A1 = np.hstack([A0, y[:, None]])
    assert o.last_step_angle_U <= 1e-12
    assert abs(o.last_step_angle_V - _angle(np.vstack([A0.T, np.zeros((1, 6))]), A1.T)) <= 1e-12
    assert abs(o.last_spectrum_change - _spec(A0, A1)) <= 1e-13


def test_entry_update_square_full_rank():
    rng = np.random.default_rng(2)
    A0 = rng.standard_normal((6, 6))
    o = OracleEngine(A0, 6, drift=True)
    o.apply(_Ev(ENTRY, i=2, j=4, delta=0.7))
    A1 = A0.copy()
    A1[2, 4] += 0.7
    assert o.last_step_angle_U <= 1e-12 and o.last_step_angle_V <= 1e-12
    assert abs(o.last_spectrum_change - _spec(A0, A1)) <= 1e-13


def test_drift_off_leaves_nan():
    o = OracleEngine(np.eye(3), 2)
    o.apply(_Ev(ROW, np.ones(3)))
    assert np.isnan(o.last_step_angle_U) and np.isnan(o.last_spectrum_change)


def test_drift_sum_bounds_the_angle_from_the_last_refresh():
    """The drift policy's quantity (Sections 3.2-3.3 surrogate): the step
    angles of U added up since the last refresh bound, by the triangle
    inequality of the largest principal angle, the angle between the span
    stored at the last refresh (zero-padded) and the current one, at every
    update of a mixed row / column run whose rank stays k."""
    from oracle import metrics
    from oracle.policies import Policy
    from synth import FactorStream
    fs = FactorStream(seed=41, stream=0, n0=30, K=5)
    A0 = fs.initial(120)
    events = fs.materialize([ROW, ROW, COL, ROW] * 12, m0=120)
    o = OracleEngine(A0, 6, policy=Policy.drift(theta_max=1e9), cgs2=True)
    U_ref = o.U.copy()
    worst = 0.0
    for ev in events:
        o.step(ev)
        assert len(o.s) == 6
        theta = metrics.theta_max(U_ref, o.U)
        assert theta <= o.drift_acc + 1e-12, (ev.t, theta, o.drift_acc)
        worst = max(worst, theta / o.drift_acc)
    assert o.n_refresh == 0 and 0.0 < worst <= 1.0


def test_drift_policy_refreshes_where_the_sum_crosses():
    """Refresh after the update at which the running sum of step angles first
    exceeds theta_max (spacing t_min); the sum restarts after each refresh,
    and a refresh restores TruncatedSVD(A_t, k)."""
    from oracle.policies import Policy
    from oracle.svd import truncated_svd
    from synth import FactorStream
    fs = FactorStream(seed=43, stream=0, n0=25, K=4)
    A0 = fs.initial(80)
    kinds = [ROW, COL, ROW, ENTRY] * 15
    events = fs.materialize(kinds, m0=80)
    probe = OracleEngine(A0, 5, drift=True, cgs2=True)
    steps = []
    for ev in events:
        probe.step(ev)
        steps.append(probe.last_step_angle_U)
    theta_max = 0.5 * sum(steps[:20])
    o = OracleEngine(A0, 5, policy=Policy.drift(theta_max=theta_max, t_min=3), cgs2=True)
    want = []
    for ev in events:
        fired = o.step(ev)
        assert o.last_step_angle_U >= 0.0
        if fired:
            want.append(ev.t)
            U, s, V = truncated_svd(o.A, 5)
            assert np.allclose(np.abs(o.s), s, rtol=0, atol=1e-12 * s[0])
            assert o.drift_acc == 0.0
    # the first refresh is the first tick whose running sum (same run until
    # then) exceeds theta_max
    first = next(i for i in range(len(steps)) if sum(steps[:i + 1]) > theta_max) + 1
    assert want and want[0] == max(first, 3), (want, first)
    assert all(b - a >= 3 for a, b in zip(want, want[1:]))
