"""Segmented refresh batches (isvd_set_segmented_refresh): the refreshes that
the policies of one tick fire (Sec. 3), for FP32 streams whose TruncatedSVD
(Sec. 2.4.1) runs in the A form, computed together with one launch per
refresh phase.  Every stream's factors, header and trackers are bitwise
those of the same refreshes run one by one on the refresh lanes, over a mix
that reaches every branch of the batch:

* one and two subspace iterations (two launch groups), and a block spanning
  all columns (no iteration);
* a block width that is not a multiple of four (CholQR's rotation off the
  matrix cores) and widths of one to six 16-column tiles;
* deferred-U streams (W and W^-1 reset by the commit) and angle-policy
  streams (reference trackers reset), next to an FP64 stream that the batch
  leaves to the lanes;
* ticks whose refreshes all go to the batch, and ticks with none for it;
* error-policy streams, whose checks (Sec. 3.2) are computed as one batch and
  whose refresh, when the ratio exceeds gamma, commits from that batch: the
  same decisions and states as the checks made one by one;
* row, column and entry updates between the refreshes."""
import numpy as np
import pytest

from synth import FactorStream, ROW, COL, ENTRY

pytestmark = pytest.mark.gpu

T = 13
# (m0, n0, k, refresh_iters, policy kind, precision)
STREAMS = [(900, 120, 16, 1, "periodic", "fp32"),     # b = 24
           (1200, 200, 32, 1, "periodic", "fp32"),    # b = 48
           (1500, 300, 64, 1, "periodic", "fp32"),    # b = 96
           (700, 40, 32, 1, "periodic", "fp32"),      # b = n: exact A form
           (800, 90, 10, 1, "periodic", "fp32"),      # b = 18
           (1000, 150, 16, 2, "periodic", "fp32"),    # two iterations
           (1100, 160, 24, 1, "angle", "fp32"),       # angle trackers
           (600, 100, 12, 1, "angle", "fp32"),        # b = 20
           (1200, 140, 16, 1, "error", "fp32"),       # checks every 3 updates
           (900, 60, 24, 2, "error", "fp32"),
           (900, 110, 16, 1, "periodic", "fp64")]     # not batched, period 5


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_24514_amd import isvd
    return torch, isvd


def _kind(s, t):
    if t % 5 == 2 and s % 2 == 0:
        return COL
    if t % 3 == 1:
        return ENTRY
    return ROW


def _run(torch, isvd, segmented):
    data = []
    for s, (m0, n0, k, it, pol, prec) in enumerate(STREAMS):
        fs = FactorStream(seed=91, stream=s, n0=n0, K=5)
        data.append((fs.initial(m0), fs.materialize([_kind(s, t) for t in range(T)], m0=m0)))
    with isvd.Engine() as eng:
        eng.set_deferred_u(True)
        eng.set_segmented_refresh(segmented)
        sids = []
        for (m0, n0, k, it, pol, prec), (A0, _) in zip(STREAMS, data):
            if pol == "periodic":
                # the FP64 stream refreshes in other ticks: ticks whose refreshes are all batched
                p = isvd.Policy(kind=isvd.POL_PERIODIC, period=4 if prec == "fp32" else 5)
            elif pol == "angle":
                p = isvd.Policy(kind=isvd.POL_ANGLE, theta_max=1e-12, t_min=4)
            else:
                p = isvd.Policy(kind=isvd.POL_ERROR, gamma=1.0, check_every=3, t_min=3)
            A = A0.astype(np.float32) if prec == "fp32" else A0
            sids.append(eng.init(A, k, prec, m_cap=m0 + T, n_cap=n0 + T, refresh_iters=it, policy=p))
        dt = {"fp32": torch.float32, "fp64": torch.float64}
        for t in range(T):
            reqs = []
            for q, (sid, (_, evs)) in enumerate(zip(sids, data)):
                ev = evs[t]
                if ev.kind == ENTRY:
                    reqs.append((sid, isvd.ENTRY, (ev.i, ev.j, ev.delta)))
                else:
                    pay = torch.tensor(ev.vec, dtype=dt[STREAMS[q][5]], device="cuda")
                    reqs.append((sid, isvd.ROW if ev.kind == ROW else isvd.COL, pay))
            eng.tick(reqs)
        torch.cuda.synchronize()
        out = []
        for sid in sids:
            met = eng.metrics(sid)
            out.append((eng.factors(sid), met))
    return out


def test_segmented_batch_is_bitwise_the_lane_refreshes(env):
    torch, isvd = env
    seg = _run(torch, isvd, True)
    lanes = _run(torch, isvd, False)
    for q, ((fa, ma), (fb, mb)) in enumerate(zip(seg, lanes)):
        print(STREAMS[q], "refreshes", ma["n_refresh"], "k", ma["k"], "angle_ref", ma["angle_ref"])
        assert ma["n_refresh"] >= (1 if STREAMS[q][4] == "error" else 2), (q, ma["n_refresh"])
        for a, b in zip(fa, fb):
            assert a.shape == b.shape and np.array_equal(a, b), q
        for key in ("t", "m", "n", "n_refresh", "t_last_refresh", "k", "status", "fro2_A", "sigma2_sum", "evr",
                    "rho", "angle_ref", "step_angle_U", "step_angle_V", "spectrum_change"):
            va, vb = ma[key], mb[key]
            assert va == vb or (va != va and vb != vb), (q, key, va, vb)
