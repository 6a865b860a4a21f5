"""Captured ticks (isvd_set_tick_graphs): a deferred-U tick of row appends
replayed from a HIP graph gives every stream the same bits as the same tick
launched directly, over enough ticks to cross the explicit-U flush points
(every m / (8 k) appends), with two request sets alternating (the graph
cache), and with the streams' row counts growing past a U-rotation tile
boundary (the captured grid is sized for the capacity)."""
import numpy as np
import pytest

from synth import FactorStream, ROW

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_24514_amd import isvd
    return torch, isvd


def test_captured_ticks_match_direct_ticks(env):
    torch, isvd = env
    ks = (8, 16, 32, 64, 128)
    shapes = [(1000 + 37 * s, (40 if ks[s % 5] < 64 else 140) + 4 * (s % 3), ks[s % 5]) for s in range(30)]
    T = 40
    data = []
    for s, (m0, n0, k) in enumerate(shapes):
        fs = FactorStream(seed=81, stream=s, n0=n0, K=5 if k < 64 else 20)
        data.append((fs.initial(m0).astype(np.float32), k, fs.materialize([ROW] * T, m0=m0)))
    res = {}
    for graphs in (True, False):
        with isvd.Engine() as eng:
            eng.set_deferred_u(True)
            eng.set_tick_graphs(graphs)
            sids = [eng.init(A0, k, "fp32", m_cap=A0.shape[0] + T, n_cap=A0.shape[1]) for A0, k, _ in data]
            pays = [[torch.tensor(ev.vec, dtype=torch.float32, device="cuda") for ev in evs] for _, _, evs in data]
            st = torch.cuda.Stream()
            for t in range(T):
                # two request sets alternate for the first half: all streams, then the even ones
                if t < T // 2 and t % 2 == 1:
                    sel = list(range(0, len(sids), 2))
                else:
                    sel = list(range(len(sids)))
                eng.tick([(sids[q], isvd.ROW, pays[q][t]) for q in sel], stream=st)
            # streams skipped on odd early ticks get their rows at the end
            for t in range(1, T // 2, 2):
                eng.tick([(sids[q], isvd.ROW, pays[q][t]) for q in range(1, len(sids), 2)], stream=st)
            st.synchronize()
            res[graphs] = [eng.factors(sid) for sid in sids]
    for q in range(len(shapes)):
        for a, b in zip(res[True][q], res[False][q]):
            assert a.shape == b.shape and np.array_equal(a, b), q
