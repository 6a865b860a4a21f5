"""Qualitative replication of the synthetic experiments of Section 4 on the
FP64 oracle, as sanity bands on this repository's generator (the paper's
generator is unspecified; its values are bands, not targets):

* E1 (Section 4.1): without refresh the Frobenius ratio of 10000 rank-1
  updates of a rank-5 50 x 40 matrix settles near 1.12; a refresh every
  1000 updates returns it to 1 each time (a sawtooth).
* E2 (Section 4.2): the no-refresh ratio rises with k in {5, 8, 12} (the
  same matrix with noise 0.1, so that every k is within the numerical rank).
* E3 (Section 4.3): rows and columns of a rank-6 model with k = 4 and a
  refresh every 50 keep the ratio within 1.0-1.02.
"""
import numpy as np

from oracle.engine import OracleEngine
from oracle.policies import Policy
from tests.experiments import E1_CHECK, e1_stream, e3_stream


def _ratios(A0, k, events, policy, every):
    o = OracleEngine(A0, k, policy=policy)
    out = []
    for q, ev in enumerate(events):
        o.step(ev)
        if (q + 1) % every == 0:
            out.append(o.exact_metrics()["frob_ratio"])
    return np.array(out)


def test_e1_drift_and_refresh_sawtooth():
    A0, ev = e1_stream()
    none = _ratios(A0, 5, ev, None, E1_CHECK)
    saw = _ratios(A0, 5, ev, Policy.periodic(1000), E1_CHECK)
    assert 1.05 <= none[-1] <= 1.2 and none.max() <= 1.25
    at_refresh = saw[(1000 // E1_CHECK) - 1::1000 // E1_CHECK]
    assert np.all(np.abs(at_refresh - 1.0) <= 1e-9)
    assert saw.mean() < none.mean() and saw.min() >= 1.0 - 1e-9


def test_e2_ratio_rises_with_k():
    A0, ev = e1_stream(4000, noise=0.1)
    ends = [_ratios(A0, k, ev, None, len(ev))[-1] for k in (5, 8, 12)]
    assert ends[0] < ends[1] < ends[2]


def test_e3_growth_with_refresh_every_50():
    A0, ev = e3_stream()
    r = _ratios(A0, 4, ev, Policy.periodic(50), 10)
    assert np.all((r >= 1.0 - 1e-9) & (r <= 1.02))
    assert abs(r[4] - 1.0) <= 1e-9 and abs(r[9] - 1.0) <= 1e-9
