"""GPU parity of the finance readout (Section 5) against the FP64 oracle.

Bars (each written in its test):
* causal de-meaning: the kernel runs the recurrence's operations in the
  oracle's order in FP64: FP64 output within 4 eps of the oracle's (relative
  to the largest return), FP32 output within one FP32 rounding of the
  oracle's value; split calls equal one call.
* covariance and volatility from the engine's own factors (pulled to the
  host exactly): 1e-12 relative (FP64 sums in a different order); the
  covariance is exactly symmetric.
* exact side (refresh block spanning all columns, so the truncated SVD is
  exact up to rounding): against the oracle's TruncatedSVD of the engine's A:
  volatility 1e-9 (FP64 storage) / 1e-5 (FP32 storage) relative, risk error
  1e-9 / 2e-5 absolute.  The covariance error comes from k x k products
  whose three squared terms are O(1) relative to ||Sigma_full||_F^2 and
  cancel down to err_cov^2: rounding of about k eps64 in them leaves
  err_cov exact to about sqrt(k eps64) = 4e-8 absolute (k = 5), so its bar
  is 2e-7 (FP64 storage) / 2e-5 (FP32 storage, the refresh's FP32
  products).
* a returns stream centred and appended on the GPU against the oracle engine
  fed the oracle's centred rows: the FP32 bars of the update tests
  (volatility and covariance 1e-5 relative).
"""
import numpy as np
import pytest

from oracle import finance as F
from oracle.engine import OracleEngine
from oracle.svd import truncated_svd
from synth import FactorStream, ROW

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def isvd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_24514_amd import isvd as mod
    return mod


def _returns(seed, t, n, K=5):
    """Factor-model rows scaled to daily-return size, plus a per-asset drift."""
    fs = FactorStream(seed=seed, stream=0, n0=n, K=K)
    drift = 0.0005 * np.random.default_rng(seed + 100).standard_normal(n)
    return 0.01 * fs.initial(t) + drift


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_causal_center_matches_oracle(isvd, dtype):
    import torch
    r = _returns(1, 300, 37)
    rt = torch.tensor(r, dtype=getattr(torch, dtype), device="cuda")
    mu = torch.zeros(37, dtype=torch.float64, device="cuda")
    a = isvd.causal_center(rt[:100], mu, 0)
    b = isvd.causal_center(rt[100:], mu, 100)
    got = torch.cat([a, b]).cpu().numpy().astype(np.float64)
    want, mu_want = F.causal_center(rt.cpu().numpy().astype(np.float64))
    scale = np.abs(r).max()
    if dtype == "float64":
        assert np.abs(got - want).max() <= 4 * 2.2e-16 * scale
    else:
        assert np.abs(got - want.astype(np.float32)).max() <= 6e-8 * np.abs(want).max()
    assert np.abs(mu.cpu().numpy() - mu_want).max() <= 4 * 2.2e-16 * scale
    assert np.array_equal(got[0], np.zeros(37))
    whole = isvd.causal_center(rt, torch.zeros(37, dtype=torch.float64, device="cuda"), 0)
    assert torch.equal(whole, torch.cat([a, b]))


def _stream(isvd, eng, precision, seed=2, t0=400, n=40, k=5, appends=30):
    R, _ = F.causal_center(_returns(seed, t0 + appends, n))
    sid = eng.init(R[:t0], k, precision, m_cap=t0 + appends, n_cap=n, oversample=64)
    for q in range(appends):
        eng.append_row(sid, R[t0 + q])
    return sid, R


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_covariance_and_volatility_from_the_engine_factors(isvd, precision):
    with isvd.Engine() as eng:
        sid, R = _stream(isvd, eng, precision)
        m = R.shape[0]
        U, S, V = eng.factors(sid)
        C = eng.covariance(sid).cpu().numpy()
        want = F.low_rank_cov(V, S, m)
        assert np.abs(C - want).max() <= 1e-12 * np.abs(want).max()
        assert np.array_equal(C, C.T)
        rng = np.random.default_rng(5)
        for w in (np.full(40, 1.0 / 40), rng.standard_normal(40), np.eye(40)[7]):
            got = eng.risk(sid, w)
            vw = F.portfolio_vol(V, S, m, w)
            assert abs(got["vol_inc"] - vw) <= 1e-12 * vw
            assert np.isnan(got["vol_full"]) and np.isnan(got["err_cov"]) and np.isnan(got["err_risk"])


@pytest.mark.parametrize("precision,rel,absb,covb", [("fp64", 1e-9, 1e-9, 2e-7), ("fp32", 1e-5, 2e-5, 2e-5)])
def test_exact_side_against_the_oracle_truncated_svd(isvd, precision, rel, absb, covb):
    with isvd.Engine() as eng:
        sid, R = _stream(isvd, eng, precision, appends=60)
        m = R.shape[0]
        U, S, V = eng.factors(sid)
        A = eng.matrix(sid)
        _, sf, Vf = truncated_svd(A, len(S))
        w = np.full(40, 1.0 / 40)
        got = eng.risk(sid, w, exact=True)
        vol_full = F.portfolio_vol(Vf, sf, m, w)
        vol_inc = F.portfolio_vol(V, S, m, w)
        err_cov = F.cov_error(V, S, Vf, sf, m)
        print(precision, got, "oracle", vol_full, err_cov)
        assert abs(got["vol_full"] - vol_full) <= rel * vol_full
        assert abs(got["err_cov"] - err_cov) <= covb
        assert abs(got["err_risk"] - F.risk_error(vol_inc, vol_full)) <= absb
        # the stream itself is unchanged by the exact readout
        U2, S2, V2 = eng.factors(sid)
        assert np.array_equal(S, S2) and np.array_equal(V, V2)


def test_returns_stream_end_to_end(isvd):
    """Returns centred on the GPU and appended (FP32 storage) against the
    oracle engine fed the oracle's centred rows."""
    import torch
    r = _returns(7, 460, 40)
    Ro, _ = F.causal_center(r)
    o = OracleEngine(Ro[:400], 5, tol_rel=1e-5, cgs2=True)
    rt = torch.tensor(r, dtype=torch.float32, device="cuda")
    mu = torch.zeros(40, dtype=torch.float64, device="cuda")
    with isvd.Engine() as eng:
        R0 = isvd.causal_center(rt[:400], mu, 0)
        sid = eng.init(R0, 5, "fp32", m_cap=460, n_cap=40, oversample=64)
        for q in range(60):
            x = isvd.causal_center(rt[400 + q], mu, 400 + q)
            eng.append_row(sid, x)
            o.step(_Row(Ro[400 + q]))
        torch.cuda.synchronize()
        w = np.full(40, 1.0 / 40)
        got = eng.risk(sid, w)["vol_inc"]
        want = F.portfolio_vol(o.V, o.s, 460, w)
        assert abs(got - want) <= 1e-5 * want
        C = eng.covariance(sid).cpu().numpy()
        Co = F.low_rank_cov(o.V, o.s, 460)
        assert np.linalg.norm(C - Co) <= 1e-5 * np.linalg.norm(Co)


class _Row:
    def __init__(self, vec):
        self.kind, self.vec = ROW, vec


def test_readout_argument_errors(isvd):
    import torch
    with isvd.Engine() as eng:
        sid, _ = _stream(isvd, eng, "fp64", appends=2)
        with pytest.raises(isvd.IsvdError) as e:
            eng.risk(sid, np.ones(39))
        assert e.value.status == -2
        bad = torch.empty((40, 39), dtype=torch.float64, device="cuda")
        with pytest.raises(isvd.IsvdError) as e:
            eng._check(eng._lib.isvd_covariance(eng._h, sid, isvd.ctypes.c_void_p(bad.data_ptr()), 39, None),
                       "isvd_covariance")
        assert e.value.status == -1
        mu = torch.zeros(5, dtype=torch.float64, device="cuda")
        with pytest.raises(isvd.IsvdError) as e:
            isvd.causal_center(torch.zeros((0, 5), dtype=torch.float64, device="cuda"), mu, 0)
        assert e.value.status == -1
