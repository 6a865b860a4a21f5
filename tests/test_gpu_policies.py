"""GPU parity of the exact metrics and of the refresh / rank policies.

* exact metrics (eq. frob-errors, eq. frob-ratio): E_inc, E_opt and the
  ratio against the oracle's on the same state; ||Q^T Q - I||_2 of the GPU's
  own factors against the same norm taken on the host.  Bars: 1e-9 relative
  in the FP64 path, 1e-5 in the FP32 path (its A is stored in FP32).
* error-threshold policy (eq. error-refresh-rule): the GPU refreshes at the
  oracle's ticks.  The test first checks that no check tick has a ratio
  within 1e-6 of gamma, so that rounding cannot flip a decision.
* adaptive rank (Section 3.4): the GPU's rank follows the oracle's tick by
  tick, shrinking on a five-factor panel and growing on novel rows.
The refresh block spans all columns here (oversample >= n), so the GPU's
TruncatedSVD and E_opt are exact like the oracle's."""
import numpy as np
import pytest

from synth import FactorStream, event_schedule_c0, ROW, COL, ENTRY
from synth.factor_model import Event
from oracle.engine import OracleEngine
from oracle.metrics import orthogonality
from oracle.policies import Policy as OPolicy
from tests.parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def isvd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_24514_amd import isvd as mod
    return mod


def _apply_gpu(eng, sid, ev):
    if ev.kind == ROW:
        eng.append_row(sid, ev.vec)
    elif ev.kind == COL:
        eng.append_col(sid, ev.vec)
    else:
        eng.update_entry(sid, ev.i, ev.j, ev.delta)


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-9), ("fp32", 1e-5)])
def test_exact_metrics_match_oracle(isvd, precision, bar):
    fs = FactorStream(seed=4, stream=0, n0=40, K=5)
    A0 = fs.initial(300)
    events = fs.materialize([ROW, ENTRY, COL, ROW, ENTRY] * 8, m0=300)
    with isvd.Engine() as eng:
        sid = eng.init(A0, 8, precision=precision, m_cap=400, n_cap=60, oversample=64)
        o = OracleEngine(A0, 8, tol_rel=1e-10 if precision == "fp64" else 1e-5, cgs2=True)
        for ev in events:
            _apply_gpu(eng, sid, ev)
            o.step(ev)
            if ev.t % 10 != 0:
                continue
            g = eng.metrics(sid, exact=True)
            x = o.exact_metrics()
            print(precision, ev.t, g["frob_error"], x["frob_error"], g["frob_opt"], x["frob_opt"])
            assert abs(g["frob_error"] - x["frob_error"]) <= bar * x["frob_error"], ev.t
            assert abs(g["frob_opt"] - x["frob_opt"]) <= bar * x["frob_opt"], ev.t
            assert abs(g["frob_ratio"] - x["frob_ratio"]) <= 2 * bar * x["frob_ratio"], ev.t
            U, S, V = eng.factors(sid)
            # the device's 2-norm of the orthogonality residual, against the host's
            assert abs(g["ortho_U"] - orthogonality(U)) <= 1e-12
            assert abs(g["ortho_V"] - orthogonality(V)) <= 1e-12
            assert g["ortho_U"] <= (1e-13 if precision == "fp64" else 1e-5)
            # a dry run: the factors did not change, no refresh was counted
            assert g["n_refresh"] == 0
            U2, S2, V2 = eng.factors(sid)
            assert np.array_equal(U, U2) and np.array_equal(S, S2)


def _c0_events():
    fs = FactorStream(seed=0, stream=0, n0=50, K=5)
    A0 = fs.initial(500)
    return A0, fs.materialize(event_schedule_c0(0, 0, 1000, 200), m0=500)


def test_error_policy_fires_at_the_oracles_ticks(isvd):
    A0, events = _c0_events()
    events = events[:400]
    gamma, every = 1.0025, 25
    o = OracleEngine(A0, 10, policy=OPolicy.error(gamma=gamma, check_every=every), cgs2=True)
    # the oracle's ratios at its check ticks keep away from gamma
    for ev in events:
        o.apply(ev)
        if ev.t % every == 0 and ev.t - o.t_last >= every:
            r = o.exact_metrics()["frob_ratio"]
            assert abs(r - gamma) > 1e-6, (ev.t, r)
        if o.decide(ev.kind):
            o.refresh(store_reference=True)
            o.refresh_ticks.append(o.t)
    assert 2 <= len(o.refresh_ticks) <= 10, o.refresh_ticks
    pol = isvd.Policy(kind=isvd.POL_ERROR, gamma=gamma, check_every=every, t_min=every)
    o2 = OracleEngine(A0, 10, cgs2=True)
    with isvd.Engine() as eng:
        sid = eng.init(A0, 10, precision="fp64", m_cap=1000, n_cap=50, oversample=64, policy=pol)
        seen = []
        for ev in events:
            _apply_gpu(eng, sid, ev)
            met = eng.metrics(sid)
            fired = met["t_last_refresh"] == ev.t and met["n_refresh"] > len(seen)
            if fired:
                seen.append(ev.t)
            o2.step(ev, force_refresh=fired)
        print("oracle", o.refresh_ticks, "gpu", seen)
        assert seen == o.refresh_ticks
        c = compare(eng.factors(sid), (o2.U, o2.s, o2.V))
        assert c["recon"] <= 1e-10, c


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("fp32", 2e-5)])
def test_adaptive_rank_shrinks_like_the_oracle(isvd, precision, bar):
    fs = FactorStream(seed=0, stream=0, n0=50, K=5)
    A0 = fs.initial(500)
    evs = fs.materialize([ROW] * 60 + [ENTRY] * 20 + [ROW] * 40, m0=500)
    opol = OPolicy.adaptive(tau=0.95, k_min=1, k_max=10, period=50)
    pol = isvd.Policy(kind=isvd.POL_ADAPTIVE, tau=0.95, band=0.01, eta=0.5, k_min=1, k_max=10, period=50)
    o = OracleEngine(A0, 10, tol_rel=1e-10 if precision == "fp64" else 1e-5, policy=opol, cgs2=True)
    with isvd.Engine() as eng:
        sid = eng.init(A0, 10, precision=precision, m_cap=700, n_cap=50, oversample=64, policy=pol)
        ks = []
        for ev in evs:
            _apply_gpu(eng, sid, ev)
            o.step(ev)
            met = eng.metrics(sid)
            ks.append(met["k"])
            assert met["k"] == len(o.s), (ev.t, met["k"], len(o.s))
            assert eng.shape(sid)[2] == len(o.s)
            if ev.t % 10 == 0:
                c = compare(eng.factors(sid), (o.U, o.s, o.V))
                assert c["recon"] <= bar, (ev.t, c)
        print(precision, "ranks", ks[:12], "...", ks[-1])
        assert ks[-1] == 4
        assert met["n_refresh"] == o.n_refresh


def test_adaptive_rank_grows_on_novel_rows(isvd):
    rng = np.random.default_rng(0)
    A0 = rng.standard_normal((40, 3)) @ rng.standard_normal((3, 30))
    opol = OPolicy.adaptive(tau=0.5, band=0.01, eta=0.5, k_min=3, k_max=6, period=0)
    pol = isvd.Policy(kind=isvd.POL_ADAPTIVE, tau=0.5, band=0.01, eta=0.5, k_min=3, k_max=6, period=0)
    o = OracleEngine(A0, 3, policy=opol, cgs2=True)
    with isvd.Engine() as eng:
        sid = eng.init(A0, 3, precision="fp64", m_cap=50, n_cap=30, oversample=64, policy=pol)
        for t in range(4):
            x = rng.standard_normal(30)
            x -= o.V @ (o.V.T @ x)
            ev = Event(ROW, t + 1, vec=x * 50.0)
            _apply_gpu(eng, sid, ev)
            o.step(ev)
            assert eng.metrics(sid)["k"] == len(o.s), t
        assert len(o.s) > 3
        c = compare(eng.factors(sid), (o.U, o.s, o.V))
        assert c["recon"] <= 1e-10, c


def test_adaptive_rank_in_batched_ticks(isvd):
    import torch
    streams = [FactorStream(seed=5, stream=q, n0=48, K=5) for q in range(3)]
    A0s = [fs.initial(400) for fs in streams]
    kinds = [ROW, ENTRY, ROW, ROW] * 12
    evs = [fs.materialize(kinds, m0=400) for fs in streams]
    opol = OPolicy.adaptive(tau=0.95, k_min=1, k_max=12, period=20)
    pol = isvd.Policy(kind=isvd.POL_ADAPTIVE, tau=0.95, band=0.01, eta=0.5, k_min=1, k_max=12, period=20)
    os_ = [OracleEngine(A0, 12, policy=opol, cgs2=True) for A0 in A0s]
    with isvd.Engine() as eng:
        sids = [eng.init(A0, 12, precision="fp64", m_cap=500, n_cap=48, oversample=64, policy=pol) for A0 in A0s]
        for t in range(len(kinds)):
            reqs = []
            for q in range(3):
                ev = evs[q][t]
                if ev.kind == ROW:
                    reqs.append((sids[q], ROW, torch.tensor(ev.vec, dtype=torch.float64, device="cuda")))
                else:
                    reqs.append((sids[q], ENTRY, (ev.i, ev.j, ev.delta)))
                os_[q].step(ev)
            eng.tick(reqs)
            for q in range(3):
                assert eng.metrics(sids[q])["k"] == len(os_[q].s), (t, q)
        for q in range(3):
            c = compare(eng.factors(sids[q]), (os_[q].U, os_[q].s, os_[q].V))
            assert c["recon"] <= 1e-10, (q, c)


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-9), ("fp32", 2e-5)])
def test_angle_trackers_match_direct_and_oracle(isvd, precision, bar):
    """theta_ref tracked through every update (rows, columns, entries) against
    the same angle formed directly on the GPU and the oracle's (Section 2.4.2),
    with a threshold that never fires."""
    fs = FactorStream(seed=6, stream=0, n0=40, K=5)
    A0 = fs.initial(300)
    evs = fs.materialize([ROW, COL, ENTRY, ROW] * 15, m0=300)
    pol = isvd.Policy(kind=isvd.POL_ANGLE, theta_max=10.0, t_min=1)
    o = OracleEngine(A0, 8, tol_rel=1e-10 if precision == "fp64" else 1e-5, cgs2=True)
    with isvd.Engine() as eng:
        sid = eng.init(A0, 8, precision=precision, m_cap=400, n_cap=80, oversample=64, policy=pol)
        assert eng.metrics(sid)["angle_ref"] == 0.0
        for ev in evs:
            _apply_gpu(eng, sid, ev)
            o.step(ev)
            if ev.t % 5 != 0:
                continue
            tracked = eng.metrics(sid)["angle_ref"]
            direct = eng.metrics(sid, exact=True)["angle_ref"]
            ref = o.angle_ref(0)
            print(precision, ev.t, tracked, direct, ref)
            assert abs(tracked - ref) <= bar, (ev.t, tracked, ref)
            assert abs(direct - ref) <= bar, (ev.t, direct, ref)
        assert eng.metrics(sid)["n_refresh"] == 0


def test_angle_policy_fires_at_the_oracles_ticks(isvd):
    A0, events = _c0_events()
    events = events[:400]
    theta_max = 2e-4
    o = OracleEngine(A0, 10, policy=OPolicy.angle(theta_max=theta_max), cgs2=True)
    # the oracle's angles keep away from the threshold
    for ev in events:
        o.apply(ev)
        if o.t - o.t_last >= 1:
            assert abs(o.angle_ref(0) - theta_max) > 1e-9, ev.t
        if o.decide(ev.kind):
            o.refresh(store_reference=True)
            o.refresh_ticks.append(o.t)
    assert 3 <= len(o.refresh_ticks) <= 20, o.refresh_ticks
    pol = isvd.Policy(kind=isvd.POL_ANGLE, theta_max=theta_max, t_min=1)
    with isvd.Engine() as eng:
        sid = eng.init(A0, 10, precision="fp64", m_cap=1000, n_cap=50, oversample=64, policy=pol)
        seen = []
        for ev in events:
            _apply_gpu(eng, sid, ev)
            met = eng.metrics(sid)
            if met["t_last_refresh"] == ev.t and met["n_refresh"] > len(seen):
                seen.append(ev.t)
                assert met["angle_ref"] == 0.0
        print("oracle", o.refresh_ticks, "gpu", seen)
        assert seen == o.refresh_ticks
