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


def test_completion_waits_for_the_tick_under_deferred_u(env):
    """With deferred U a tick's work ends on the server's stream, not on the
    rotation lane: a completion the server reports must find that stream
    idle (nothing else was queued on it after the tick)."""
    torch, isvd = env
    nst, m0, n0, k = 24, 20000, 600, 64
    st = torch.cuda.Stream()
    with isvd.Engine() as eng:
        eng.set_deferred_u(True)
        with isvd.Server(eng, max_inflight=4, stream=st) as srv:
            tickets = []
            for s in range(nst):
                A0 = torch.randn((m0, n0), generator=torch.Generator(device="cuda").manual_seed(100 + s),
                                 device="cuda", dtype=torch.float32)
                tickets.append(srv.add_stream(A0, k, m_cap=m0 + 8, n_cap=n0, oversample=96))
            rows = [torch.randn(n0, device="cuda", dtype=torch.float32) for _ in range(nst)]
            # admit and initialise every stream first
            t0 = srv.clock()
            for s in range(nst):
                srv.submit(tickets[s], ROW, rows[s], t0)
            while srv.stats()["queued"] > 0:
                srv.step()
            srv.drain()
            srv.poll()
            st.synchronize()
            # one tick of nst row appends, then poll without blocking
            t0 = srv.clock()
            for s in range(nst):
                srv.submit(tickets[s], ROW, rows[s], t0)
            srv.step()
            seen = []
            for _ in range(200_000):
                srv.step()                  # nothing queued: only stamps finished ticks
                seen = srv.poll()
                if seen:
                    break
            assert seen, "no completion"
            assert st.query(), "completion reported while the tick still ran on the server's stream"
            srv.drain()


def test_stream_with_a_rejected_request_retires(env):
    """A request that completes with an error still counts toward the
    stream's lifetime, so the stream retires and frees its budget for the
    next one (FIFO admission would otherwise stall)."""
    torch, isvd = env
    data = _workload(3, seed=14)
    (A0, k, evs), (B0, kb, evb) = data[0], data[1]
    with isvd.Engine() as eng:
        ca = isvd.Engine.config(A0.shape[0], A0.shape[1], k, "fp32", m_cap=A0.shape[0] + 4, n_cap=A0.shape[1] + 4,
                                oversample=96)
        cb = isvd.Engine.config(B0.shape[0], B0.shape[1], kb, "fp32", m_cap=B0.shape[0] + 4, n_cap=B0.shape[1] + 4,
                                oversample=96)
        budget = max(eng.stream_bytes(ca), eng.stream_bytes(cb))      # one stream at a time
        with isvd.Server(eng, hbm_budget=budget) as srv:
            ta = srv.add_stream(torch.tensor(A0, dtype=torch.float32, device="cuda"), k, m_cap=A0.shape[0] + 4,
                                n_cap=A0.shape[1] + 4, lifetime=2, oversample=96)
            tb = srv.add_stream(torch.tensor(B0, dtype=torch.float32, device="cuda"), kb, m_cap=B0.shape[0] + 4,
                                n_cap=B0.shape[1] + 4, lifetime=1, oversample=96)
            bad = torch.zeros(A0.shape[1] + 3, dtype=torch.float32, device="cuda")
            good = torch.tensor(FactorStream(seed=12, stream=0, n0=A0.shape[1], K=5).row(A0.shape[0], A0.shape[1]),
                                dtype=torch.float32, device="cuda")
            t0 = srv.clock()
            srv.submit(ta, ROW, bad, t0)
            srv.submit(ta, ROW, good, t0)
            srv.submit(tb, ENTRY, (0, 0, 0.5), t0)
            for _ in range(1000):
                srv.step()
                if srv.stats()["retired"] == 2:
                    break
            srv.drain()
            comp = sorted(srv.poll(), key=lambda c: c["req"])
            assert srv.stats()["retired"] == 2
            assert [c["status"] for c in comp] == [-2, 0, 0]
