"""GPU parity of the drift signals of each update (the surrogates of the
error- and angle-based refresh, Sections 3.2-3.3) against the FP64 oracle,
which forms them by definition (principal angles of the bases before and
after, the spectrum's relative change).

Bars: FP64 storage 1e-9 absolute on the angles (radians) and on the
spectrum change (both sides in FP64, states within 1e-12 of each other);
FP32 storage 2e-5 absolute (the FP32 states differ from the oracle's by
about 1e-6 relative).  Entry updates keep both spans, so the engine reports
angle 0 exactly.
"""
import numpy as np
import pytest

from oracle.engine import OracleEngine
from synth import FactorStream, ROW, COL, ENTRY

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


def _close(met, o, bar, where):
    for key, want in (("step_angle_U", o.last_step_angle_U), ("step_angle_V", o.last_step_angle_V),
                      ("spectrum_change", o.last_spectrum_change)):
        assert abs(met[key] - want) <= bar, (where, key, met[key], want)


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-9), ("fp32", 2e-5)])
def test_single_stream_every_update(isvd, precision, bar):
    fs = FactorStream(seed=61, stream=0, n0=40, K=5)
    m0 = 400
    A0 = fs.initial(m0)
    kinds = [ROW] * 12 + [COL] * 3 + [ENTRY] * 2 + [ROW] * 5
    events = fs.materialize(kinds, m0=m0)
    o = OracleEngine(A0, 8, tol_rel=1e-5, cgs2=True, drift=True)
    with isvd.Engine() as eng:
        sid = eng.init(A0, 8, precision, m_cap=m0 + 20, n_cap=44, oversample=64)
        met = eng.metrics(sid)
        assert np.isnan(met["step_angle_U"]) and np.isnan(met["spectrum_change"])
        for q, ev in enumerate(events):
            _apply(eng, sid, ev)
            o.step(ev)
            met = eng.metrics(sid)
            _close(met, o, bar, (q, ev.kind))
            if ev.kind == ENTRY:
                assert met["step_angle_U"] == 0.0 and met["step_angle_V"] == 0.0
            else:
                assert met["step_angle_U"] > 0.0


def test_batched_deferred_ticks(isvd):
    """Streams over the four rank buckets, deferred U, row-append ticks: the
    signals of each stream's last update against the oracle's."""
    import torch
    ks = (8, 16, 32, 64)
    shapes = [(1500 + 300 * s, min(ks[s % 4] + 56, 72) + s % 3, ks[s % 4]) for s in range(8)]
    T = 6
    data = []
    for s, (m0, n0, k) in enumerate(shapes):
        fs = FactorStream(seed=67, stream=s, n0=n0, K=5)
        data.append((fs.initial(m0), k, fs.materialize([ROW] * T, m0=m0)))
    with isvd.Engine() as eng:
        eng.set_deferred_u(True)
        sids = [eng.init(A0, k, "fp32", m_cap=A0.shape[0] + T, n_cap=A0.shape[1], oversample=64)
                for A0, k, _ in data]
        pays = [[torch.tensor(ev.vec, dtype=torch.float32, device="cuda") for ev in evs] for _, _, evs in data]
        for t in range(T):
            eng.tick([(sid, isvd.ROW, pays[q][t]) for q, sid in enumerate(sids)])
        mets = [eng.metrics(sid) for sid in sids]
    for q, (A0, k, evs) in enumerate(data):
        o = OracleEngine(A0, k, tol_rel=1e-5, cgs2=True, drift=True)
        for ev in evs:
            o.step(ev)
        _close(mets[q], o, 2e-5, (q, k))
