"""Ranks above 64: the 65..128 bucket (k = 80, 96, 128) against the FP64
oracle (Alg. A1-A3 and TruncatedSVD, Sec. 2.4.1).

* initial SVD (Gram form, block b = min(k + k / 2, 128) < n: at k = 128 the
  block equals k, and the locked factor directions plus the refilled block
  give the oversampling) and 24 mixed updates -- rows, columns, entries --
  to the FP64 (reconstruction <= 1e-10, sigma <= 1e-12) and FP32 bars
  (2e-5, 1e-5), principal angles <= 1e-4 rad on the gap-separated scope;
  the core is of order 129 (FP64: rotations accumulated in global memory);
* a tick holding a rank-128 stream beside narrower ones gives each stream
  the same bits as its own single-stream updates;
* the BF16 rotation option at k = 128 drifts at the BF16 level and a refresh
  restores FP32 accuracy;
* theta_ref (Sec. 2.4.2) tracked through updates at k = 128 against the
  directly formed angle and the oracle's.
The panels have 40 factors (the precision-sweep workload's), n = 220.
"""
import numpy as np
import pytest

from synth import FactorStream, ROW, COL, ENTRY
from oracle.engine import OracleEngine
from oracle.svd import truncated_svd
from tests.parity import compare

pytestmark = pytest.mark.gpu

M0, N0, NF = 1600, 220, 40
KINDS = [ROW, ROW, ENTRY, COL, ROW, ENTRY, ROW, ROW] * 3


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


def _bars(precision):
    return (1e-10, 1e-12) if precision == "fp64" else (2e-5, 1e-5)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("k", [80, 96, 128])
def test_wide_rank_updates_match_the_oracle(isvd, k, precision):
    fs = FactorStream(seed=71, stream=k, n0=N0, K=NF)
    A0 = fs.initial(M0)
    if precision == "fp32":
        A0 = A0.astype(np.float32).astype(np.float64)
    events = fs.materialize(KINDS, m0=M0)
    rb, sb = _bars(precision)
    with isvd.Engine() as eng:
        sid = eng.init(A0.astype(np.float32) if precision == "fp32" else A0, k, precision,
                       m_cap=M0 + 30, n_cap=N0 + 6)
        print("case", k, precision, flush=True)
        c0 = compare(eng.factors(sid), truncated_svd(A0, k))
        print("init", c0)
        assert eng.metrics(sid)["refresh_converged"] == 1
        assert c0["recon"] <= rb and c0["sigma"] <= sb, c0
        o = OracleEngine(A0, k, tol_rel=1e-10 if precision == "fp64" else 1e-5, cgs2=True)
        for ev in events:
            _apply(eng, sid, ev)
            o.step(ev)
        c = compare(eng.factors(sid), (o.U, o.s, o.V))
        print("updates", c)
        assert c["recon"] <= rb and c["sigma"] <= sb, c
        assert c["angle_U"] <= 1e-4 and c["angle_V"] <= 1e-4, c
        assert c["ortho_U"] <= (1e-11 if precision == "fp64" else 1e-5), c


def test_rank128_in_a_mixed_tick_is_bitwise_its_own(isvd):
    import torch
    shapes = [(1200, 200, 128), (900, 150, 100), (800, 60, 16), (1000, 140, 64)]
    T = 6
    data = []
    for s, (m0, n0, k) in enumerate(shapes):
        fs = FactorStream(seed=73, stream=s, n0=n0, K=NF if k > 64 else 5)
        data.append((fs.initial(m0).astype(np.float32), k, fs.materialize([ROW] * T, m0=m0)))
    res = {}
    for mixed in (True, False):
        with isvd.Engine() as eng:
            sids = [eng.init(A0, k, "fp32", m_cap=A0.shape[0] + T, n_cap=A0.shape[1]) for A0, k, _ in data]
            pays = [[torch.tensor(ev.vec, dtype=torch.float32, device="cuda") for ev in evs] for _, _, evs in data]
            for t in range(T):
                if mixed:
                    eng.tick([(sid, isvd.ROW, pays[q][t]) for q, sid in enumerate(sids)])
                else:
                    for q, sid in enumerate(sids):
                        eng.append_row(sid, pays[q][t])
            res[mixed] = [eng.factors(sid) for sid in sids]
    for q in range(len(shapes)):
        for a, b in zip(res[True][q], res[False][q]):
            assert np.array_equal(a, b), q


def test_bf16_rotations_at_rank128(isvd):
    fs = FactorStream(seed=75, stream=0, n0=N0, K=NF)
    A0 = fs.initial(M0).astype(np.float32).astype(np.float64)
    events = fs.materialize([ROW, ROW, COL, ENTRY, ROW] * 4, m0=M0)
    k = 128
    o = OracleEngine(A0, k, tol_rel=1e-5, cgs2=True)
    with isvd.Engine() as eng:
        sb = eng.init(A0.astype(np.float32), k, "bf16rot", m_cap=M0 + 30, n_cap=N0 + 6)
        sf = eng.init(A0.astype(np.float32), k, "fp32", m_cap=M0 + 30, n_cap=N0 + 6)
        for ev in events:
            _apply(eng, sb, ev)
            _apply(eng, sf, ev)
            o.step(ev)
        cb = compare(eng.factors(sb), (o.U, o.s, o.V))
        cf = compare(eng.factors(sf), (o.U, o.s, o.V))
        print("bf16", cb)
        print("fp32", cf)
        assert cf["recon"] <= 2e-5
        assert cb["recon"] <= 3e-2 and cb["sigma"] <= 3e-2
        assert cb["recon"] > cf["recon"]
        eng.refresh(sb)
        o.refresh()
        cr = compare(eng.factors(sb), (o.U, o.s, o.V))
        print("bf16 after refresh", cr)
        assert cr["recon"] <= 2e-5 and cr["sigma"] <= 1e-5, cr


def test_angle_trackers_at_rank128(isvd):
    fs = FactorStream(seed=77, stream=0, n0=N0, K=NF)
    A0 = fs.initial(M0)
    evs = fs.materialize([ROW, COL, ENTRY, ROW] * 5, m0=M0)
    k = 128
    pol = isvd.Policy(kind=isvd.POL_ANGLE, theta_max=10.0, t_min=1)
    o = OracleEngine(A0, k, tol_rel=1e-10, cgs2=True)
    with isvd.Engine() as eng:
        sid = eng.init(A0, k, precision="fp64", m_cap=M0 + 30, n_cap=N0 + 10, policy=pol)
        for ev in evs:
            _apply(eng, sid, ev)
            o.step(ev)
            if ev.t % 5 != 0:
                continue
            tracked = eng.metrics(sid)["angle_ref"]
            direct = eng.metrics(sid, exact=True)["angle_ref"]
            ref = o.angle_ref(0)
            print(ev.t, tracked, direct, ref)
            assert abs(tracked - ref) <= 1e-9 and abs(direct - ref) <= 1e-9, (ev.t, tracked, direct, ref)
