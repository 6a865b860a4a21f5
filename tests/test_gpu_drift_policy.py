"""The drift-surrogate refresh (Sections 3.2-3.3; policy ISVD_POL_DRIFT): the
step angles of U the cores form without A, added up since the last refresh,
trigger the refresh once they exceed theta_max.  Against the oracle's policy
on the same mixed stream (FP64 storage): the same refresh ticks (the test
first checks that no decision lies within 1e-7 rad of theta_max), the summed
angle to 1e-9 rad, and the final state to the FP64 bars.

A kept in pinned host memory (a_on_host, for streams that refresh rarely):
the same kernels read and write it over the host link, so every result is
bitwise the one with A in HBM, and the stream's device footprint drops by
A's bytes."""
import numpy as np
import pytest

from synth import FactorStream, ROW, COL, ENTRY
from oracle.engine import OracleEngine
from oracle.policies import Policy
from tests.parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def isvd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_24514_amd import isvd as mod
    return mod


def _apply(eng, sid, ev):
    if ev.kind == ROW:
        eng.append_row(sid, ev.vec)
    elif ev.kind == COL:
        eng.append_col(sid, ev.vec)
    else:
        eng.update_entry(sid, ev.i, ev.j, ev.delta)


def test_drift_policy_follows_the_oracle(isvd):
    fs = FactorStream(seed=61, stream=0, n0=60, K=5)
    A0 = fs.initial(400)
    kinds = [ROW, ROW, COL, ENTRY, ROW] * 24
    events = fs.materialize(kinds, m0=400)
    k, t_min = 8, 2
    probe = OracleEngine(A0, k, drift=True, cgs2=True)
    steps = []
    for ev in events:
        probe.step(ev)
        steps.append(probe.last_step_angle_U)
    theta_max = 0.3 * float(np.sum(steps[:40]))
    o = OracleEngine(A0, k, tol_rel=1e-10, policy=Policy.drift(theta_max=theta_max, t_min=t_min), cgs2=True)
    margins = []
    for ev in events:
        t_last, acc = o.t_last, o.drift_acc
        o.step(ev)
        if o.t - t_last >= t_min:   # the policy compared acc + this step with theta_max
            margins.append(abs(acc + o.last_step_angle_U - theta_max))
    assert len(o.refresh_ticks) >= 2 and min(margins) > 1e-7, (o.refresh_ticks, min(margins))
    pol = isvd.Policy(kind=isvd.POL_DRIFT, theta_max=theta_max, t_min=t_min)
    with isvd.Engine() as eng:
        sid = eng.init(A0, k, "fp64", m_cap=500, n_cap=100, oversample=64, policy=pol)
        seen, last = [], 0
        for ev in events:
            _apply(eng, sid, ev)
            met = eng.metrics(sid)
            if met["n_refresh"] > last:
                seen.append(ev.t)
                last = met["n_refresh"]
        print("drift refreshes", seen, "oracle", o.refresh_ticks, "theta_max", theta_max)
        assert seen == o.refresh_ticks
        assert abs(eng.metrics(sid)["drift_U"] - o.drift_acc) <= 1e-9
        c = compare(eng.factors(sid), (o.U, o.s, o.V))
        assert c["recon"] <= 1e-10 and c["sigma"] <= 1e-12, c


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_a_on_host_is_bitwise_the_hbm_stream(isvd, precision):
    fs = FactorStream(seed=63, stream=0, n0=300, K=5)
    A0 = fs.initial(2000)
    events = fs.materialize([ROW, ROW, COL, ENTRY, ROW, ENTRY] * 4, m0=2000)
    a_in = A0.astype(np.float32) if precision == "fp32" else A0
    with isvd.Engine() as eng:
        sids = [eng.init(a_in, 16, precision, m_cap=2030, n_cap=310, a_on_host=h) for h in (False, True)]
        for ev in events:
            for sid in sids:
                _apply(eng, sid, ev)
        f0, f1 = eng.factors(sids[0]), eng.factors(sids[1])
        for a, b in zip(f0, f1):
            assert np.array_equal(a, b)
        assert np.array_equal(eng.matrix(sids[0]), eng.matrix(sids[1]))
        m0, m1 = eng.metrics(sids[0], exact=True), eng.metrics(sids[1], exact=True)
        for key in ("frob_error", "frob_opt", "frob_ratio", "ortho_U"):
            assert m0[key] == m1[key], key
        for sid in sids:
            eng.refresh(sid)
        for a, b in zip(eng.factors(sids[0]), eng.factors(sids[1])):
            assert np.array_equal(a, b)
        cfg_dev = eng.config(2000, 300, 16, precision, 2030, 310)
        cfg_host = eng.config(2000, 300, 16, precision, 2030, 310, a_on_host=True)
        esz = 4 if precision == "fp32" else 8
        assert eng.stream_bytes(cfg_dev) - eng.stream_bytes(cfg_host) >= esz * 2030 * 300
