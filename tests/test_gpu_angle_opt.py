"""theta_opt (the angle metric to the optimal subspace, Section 3.3): the
largest principal angle between span(U_t) and the leading left singular
vectors of A_t, as many as the model's rank.  The exact metrics form it from
the refresh they compute (U_opt = Q_Y W, never stored) and U_t; compared
with the oracle's by definition (a full SVD of A_t and the principal angles
of the two bases) after mixed updates, with the refresh block spanning all
columns (A form) and narrower than A (Gram form): 1e-9 rad in FP64 storage;
right after a refresh the angle is at the square root of rounding (the
cosine form of the angle, as for theta_ref)."""
import numpy as np
import pytest

from synth import FactorStream, ROW, COL, ENTRY
from oracle.engine import OracleEngine

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def isvd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_24514_amd import isvd as mod
    return mod


@pytest.mark.parametrize("m0,n0,K,k,oversample", [(600, 50, 5, 8, 64), (4000, 300, 20, 24, -1)])
def test_angle_opt_matches_the_oracle(isvd, m0, n0, K, k, oversample):
    fs = FactorStream(seed=65, stream=k, n0=n0, K=K)
    A0 = fs.initial(m0)
    events = fs.materialize([ROW, ROW, COL, ENTRY, ROW, ENTRY] * 5, m0=m0)
    o = OracleEngine(A0, k, tol_rel=1e-10, cgs2=True)
    with isvd.Engine() as eng:
        sid = eng.init(A0, k, "fp64", m_cap=m0 + 20, n_cap=n0 + 10, oversample=oversample)
        for q, ev in enumerate(events):
            if ev.kind == ROW:
                eng.append_row(sid, ev.vec)
            elif ev.kind == COL:
                eng.append_col(sid, ev.vec)
            else:
                eng.update_entry(sid, ev.i, ev.j, ev.delta)
            o.step(ev)
            if q % 10 == 9:
                got = eng.metrics(sid, exact=True)["angle_opt"]
                want = o.exact_metrics(with_angles=True)["angle_opt"]
                print(ev.t, got, want)
                assert abs(got - want) <= 1e-9, (ev.t, got, want)
        eng.refresh(sid)
        # the cosine form resolves angles near zero to about the square root of rounding
        assert eng.metrics(sid, exact=True)["angle_opt"] <= 1e-6
