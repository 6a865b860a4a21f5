"""Batched ticks: many streams of different (m, n, k) per launch sequence.

Each stream is checked against its own FP64 oracle run (FP32 bar 2e-5), and
a stream's result is bitwise the same alone, inside a mixed tick, and through
the single-stream entry points: the kernels' per-stream work and reduction
order do not depend on what else is in the batch."""
import numpy as np
import pytest

from synth import FactorStream, ROW, COL, ENTRY
from oracle.engine import OracleEngine
from tests.parity import compare

pytestmark = pytest.mark.gpu

SHAPES = [(300, 40, 8), (500, 60, 16), (200, 30, 5), (400, 90, 32), (350, 48, 10), (260, 36, 12)]


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_24514_amd import isvd
    return torch, isvd


def _streams(ticks, kinds_for):
    out = []
    for s, (m0, n0, k) in enumerate(SHAPES):
        fs = FactorStream(seed=5, stream=s, n0=n0, K=5)
        A0 = fs.initial(m0)
        evs = fs.materialize([kinds_for(s, t) for t in range(ticks)], m0=m0)
        out.append((A0, k, evs))
    return out


def _req(torch, isvd, sid, ev):
    if ev.kind == ENTRY:
        return (sid, isvd.ENTRY, (ev.i, ev.j, ev.delta))
    t = torch.tensor(ev.vec, dtype=torch.float32, device="cuda")
    return (sid, isvd.ROW if ev.kind == ROW else isvd.COL, t)


def test_mixed_tick_matches_oracles_and_is_batch_invariant(env):
    torch, isvd = env
    T = 24
    kinds = lambda s, t: COL if (t % 7 == 3 and s % 2 == 0) else ENTRY if (t % 5 == 4) else ROW
    streams = _streams(T, kinds)
    with isvd.Engine() as mix, isvd.Engine() as alone, isvd.Engine() as single:
        sids, orcs = [], []
        for A0, k, evs in streams:
            m0, n0 = A0.shape
            sids.append(mix.init(A0, k, "fp32", m_cap=m0 + T, n_cap=n0 + T, oversample=96))
            orcs.append(OracleEngine(A0, k, tol_rel=1e-5, cgs2=True))
        A0, k, evs0 = streams[3]
        sa = alone.init(A0, k, "fp32", m_cap=A0.shape[0] + T, n_cap=A0.shape[1] + T, oversample=96)
        ss = single.init(A0, k, "fp32", m_cap=A0.shape[0] + T, n_cap=A0.shape[1] + T, oversample=96)
        for t in range(T):
            reqs = [_req(torch, isvd, sid, evs[t]) for sid, (_, _, evs) in zip(sids, streams)]
            mix.tick(reqs)
            alone.tick([_req(torch, isvd, sa, evs0[t])])
            ev = evs0[t]
            if ev.kind == ROW:
                single.append_row(ss, torch.tensor(ev.vec, dtype=torch.float32, device="cuda"))
            elif ev.kind == COL:
                single.append_col(ss, torch.tensor(ev.vec, dtype=torch.float32, device="cuda"))
            else:
                single.update_entry(ss, ev.i, ev.j, ev.delta)
            for o, (_, _, evs) in zip(orcs, streams):
                o.step(evs[t])
        torch.cuda.synchronize()
        for q, (sid, o) in enumerate(zip(sids, orcs)):
            c = compare(mix.factors(sid), (o.U, o.s, o.V))
            print(SHAPES[q], c)
            assert c["recon"] <= 2e-5, (q, c)
            assert c["sigma"] <= 1e-5, (q, c)
            assert c["angle_U"] <= 1e-4 and c["angle_V"] <= 1e-4, (q, c)
            met = mix.metrics(sid)
            assert (met["m"], met["n"]) == o.A.shape and met["t"] == T
        Um, Sm, Vm = mix.factors(sids[3])
        Ua, Sa, Va = alone.factors(sa)
        Us, Ss, Vs = single.factors(ss)
        assert np.array_equal(Um, Ua) and np.array_equal(Sm, Sa) and np.array_equal(Vm, Va)
        assert np.array_equal(Um, Us) and np.array_equal(Sm, Ss) and np.array_equal(Vm, Vs)
        assert np.array_equal(mix.matrix(sids[3]), alone.matrix(sa))


def test_tick_validation_rejects_whole_tick(env):
    torch, isvd = env
    fs = FactorStream(seed=6, stream=0, n0=20, K=3)
    with isvd.Engine() as eng:
        a = eng.init(fs.initial(50), 4, "fp32", m_cap=60, n_cap=20, oversample=32)
        b = eng.init(fs.initial(40), 4, "fp32", m_cap=60, n_cap=20, oversample=32)
        good = torch.ones(20, dtype=torch.float32, device="cuda")
        bad = torch.ones(19, dtype=torch.float32, device="cuda")
        with pytest.raises(isvd.IsvdError) as e:
            eng.tick([(a, isvd.ROW, good), (b, isvd.ROW, bad)])
        assert e.value.status == -2
        with pytest.raises(isvd.IsvdError) as e:
            eng.tick([(a, isvd.ROW, good), (a, isvd.ROW, good)])
        assert e.value.status == -1
        assert eng.metrics(a)["t"] == 0 and eng.metrics(b)["t"] == 0


def test_rotation_block_shapes_give_identical_results(env):
    """Every autotuner candidate of the FP32 rotation does each row's
    arithmetic in the same order, so results are bitwise equal across them;
    the rows cover several blocks of every shape and a ragged last tile."""
    torch, isvd = env
    T = 6
    shapes = [(2500, 40, 8), (2100, 50, 16), (1700, 60, 32), (3000, 70, 64), (2049, 33, 20)]
    kinds = [ROW, COL, ENTRY, ROW, COL, ROW]
    data = []
    for s, (m0, n0, k) in enumerate(shapes):
        fs = FactorStream(seed=8, stream=s, n0=n0, K=5)
        data.append((fs.initial(m0), k, fs.materialize(kinds, m0=m0)))
    results = []
    for variant in range(len(isvd.ROT_VARIANTS)):
        with isvd.Engine() as eng:
            for kc in (8, 16, 32, 64):
                eng.set_rotation_variant(kc, variant)
            sids = [eng.init(A0, k, "fp32", m_cap=A0.shape[0] + T, n_cap=A0.shape[1] + T, oversample=8)
                    for A0, k, _ in data]
            for t in range(T):
                eng.tick([_req(torch, isvd, sid, evs[t]) for sid, (_, _, evs) in zip(sids, data)])
            results.append([eng.factors(sid) for sid in sids])
    for variant in range(1, len(results)):
        for q in range(len(shapes)):
            for a, b in zip(results[0][q], results[variant][q]):
                assert np.array_equal(a, b), (variant, q)
