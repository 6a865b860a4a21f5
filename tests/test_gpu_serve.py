"""Serving loop: continuous batching, HBM-budget admission, latency stamps.

* every stream's result is the same when served in a mix of streams with
  random (Poisson) arrivals as when its requests run alone, one tick each
  (bitwise: the tick kernels' per-stream arithmetic does not depend on the
  batch), and within 2e-5 (reconstruction) of the FP64 oracle;
* under a budget that holds only some streams, streams are admitted in FIFO
  order as earlier ones retire, the admitted footprint never exceeds the
  budget, and every request completes, in per-stream submission order;
* a request that no longer fits its stream completes with ISVD_E_SHAPE."""
import numpy as np
import pytest

from synth import FactorStream, ROW, COL, ENTRY
from oracle.engine import OracleEngine
from tests.parity import compare

pytestmark = pytest.mark.gpu

SHAPES = [(400, 40, 8), (600, 60, 12), (300, 30, 4), (800, 80, 20), (500, 50, 16), (700, 35, 6)]


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_24514_amd import isvd
    return torch, isvd


def _workload(nreq, seed=11):
    rng = np.random.default_rng(seed)
    out = []
    for s, (m0, n0, k) in enumerate(SHAPES):
        fs = FactorStream(seed=12, stream=s, n0=n0, K=5)
        kinds = list(rng.choice([ROW, COL, ENTRY], size=nreq, p=[0.7, 0.15, 0.15]))
        out.append((fs.initial(m0), k, fs.materialize(kinds, m0=m0)))
    return out


def _payload(torch, ev):
    if ev.kind == ENTRY:
        return (ev.i, ev.j, ev.delta)
    return torch.tensor(ev.vec, dtype=torch.float32, device="cuda")


def _poisson_order(rng, nstreams, nreq, rate):
    """(arrival time, stream, index) of every request, each stream a Poisson process."""
    items = []
    for s in range(nstreams):
        t = np.cumsum(rng.exponential(1.0 / rate, size=nreq))
        items += [(float(t[q]), s, q) for q in range(nreq)]
    return sorted(items)


def test_results_are_the_same_alone_and_in_the_mix(env):
    torch, isvd = env
    nreq = 14
    data = _workload(nreq)
    pays = [[_payload(torch, ev) for ev in evs] for (_, _, evs) in data]
    order = _poisson_order(np.random.default_rng(3), len(data), nreq, rate=2000.0)
    with isvd.Engine() as eng, isvd.Engine() as solo:
        with isvd.Server(eng, max_inflight=2) as srv:
            A0s = [torch.tensor(A0, dtype=torch.float32, device="cuda") for (A0, _, _) in data]
            tickets = [srv.add_stream(A0s[s], k, m_cap=A0.shape[0] + nreq, n_cap=A0.shape[1] + nreq, oversample=96)
                       for s, (A0, k, _) in enumerate(data)]
            t0 = srv.clock()
            for i, (ta, s, q) in enumerate(order):
                srv.submit(tickets[s], data[s][2][q].kind, pays[s][q], t0 + ta)
                if i % 5 == 4:
                    srv.step()
            while srv.stats()["queued"] > 0:
                srv.step()
            srv.drain()
            comp = srv.poll()
            assert len(comp) == len(order) and all(c["status"] == 0 for c in comp)
            assert all(c["done_s"] >= c["launch_s"] >= c["arrival_s"] - 1e-9 for c in comp)
            sids = [srv.stream(t)[0] for t in tickets]
            # alone: same requests, one per tick, on a separate engine
            for s, (A0, k, evs) in enumerate(data):
                sid = solo.init(A0s[s], k, "fp32", m_cap=A0.shape[0] + nreq, n_cap=A0.shape[1] + nreq, oversample=96)
                o = OracleEngine(A0, k, tol_rel=1e-5, cgs2=True)
                for q, ev in enumerate(evs):
                    solo.tick([(sid, ev.kind, pays[s][q])])
                    o.step(ev)
                mixed, alone = eng.factors(sids[s]), solo.factors(sid)
                for a, b in zip(mixed, alone):
                    assert np.array_equal(a, b), s
                c = compare(mixed, (o.U, o.s, o.V))
                assert c["recon"] <= 2e-5, (s, c)


def test_admission_under_a_budget_and_retirement(env):
    torch, isvd = env
    nreq = 8
    data = _workload(nreq, seed=12)
    pays = [[_payload(torch, ev) for ev in evs] for (_, _, evs) in data]
    with isvd.Engine() as eng:
        cfgs = [isvd.Engine.config(A0.shape[0], A0.shape[1], k, "fp32", m_cap=A0.shape[0] + nreq,
                                   n_cap=A0.shape[1] + nreq, oversample=96) for (A0, k, _) in data]
        sizes = [eng.stream_bytes(c) for c in cfgs]
        budget = sum(sorted(sizes)[-2:])          # room for about two streams at a time
        with isvd.Server(eng, hbm_budget=budget, max_inflight=2) as srv:
            A0s = [torch.tensor(A0, dtype=torch.float32, device="cuda") for (A0, _, _) in data]
            tickets = [srv.add_stream(A0s[s], k, m_cap=A0.shape[0] + nreq, n_cap=A0.shape[1] + nreq,
                                      lifetime=nreq, oversample=96) for s, (A0, k, _) in enumerate(data)]
            t0 = srv.clock()
            for s in range(len(data)):
                for q, ev in enumerate(data[s][2]):
                    srv.submit(tickets[s], ev.kind, pays[s][q], t0)
            comp = []
            for _ in range(10000):
                srv.step()
                st = srv.stats()
                assert st["hbm_used"] <= budget
                comp += srv.poll()
                if st["retired"] == len(data):
                    break
            srv.drain()
            comp += srv.poll()
            assert srv.stats()["retired"] == len(data)
            assert len(comp) == len(data) * nreq and all(c["status"] == 0 for c in comp)
            admit = {}
            for c in comp:
                admit[c["ticket"]] = c["admit_s"]
            assert [admit[t] for t in tickets] == sorted(admit[t] for t in tickets)   # FIFO admission
            for t in tickets:
                reqs = [c["req"] for c in comp if c["ticket"] == t]
                assert reqs == sorted(reqs)


def test_mismatched_request_completes_with_shape_error(env):
    torch, isvd = env
    data = _workload(2, seed=13)
    A0, k, evs = data[0]
    with isvd.Engine() as eng, isvd.Server(eng) as srv:
        A0d = torch.tensor(A0, dtype=torch.float32, device="cuda")
        t = srv.add_stream(A0d, k, m_cap=A0.shape[0] + 4, n_cap=A0.shape[1] + 4, oversample=96)
        bad = torch.zeros(A0.shape[1] + 3, dtype=torch.float32, device="cuda")
        srv.submit(t, ROW, bad, srv.clock())
        srv.submit(t, ROW, torch.tensor(FactorStream(seed=12, stream=0, n0=A0.shape[1], K=5).row(A0.shape[0], A0.shape[1]),
                                         dtype=torch.float32, device="cuda"), srv.clock())
        while srv.stats()["queued"] > 0:
            srv.step()
        srv.drain()
        comp = sorted(srv.poll(), key=lambda c: c["req"])
        assert [c["status"] for c in comp] == [-2, 0]
