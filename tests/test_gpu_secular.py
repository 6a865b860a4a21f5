"""GPU parity of the append core's secular-equation path (FP32 storage, rank
buckets up to 64) in the cases that take its special branches, against the
FP64 oracle started from the same exact factors.

The append core K = [[diag(s), 0], [p^T, rho]] (Alg. A1; Alg. A2 on the
transpose) has K^T K = diag(s^2, 0) + w w^T with w = [p; rho].  Exact
factors given to the engine make that structure exact too:
* repeated singular values give equal poles, merged by a rotation;
* coordinate-vector bases give exactly zero weights, which deflate;
* a payload orthogonal to the basis leaves rho as the only weight;
* a spectrum spanning more than 1e4 sends the core back to Jacobi sweeps.
The bar is the FP32 one of the other update tests: reconstruction <= 2e-5
relative, singular values <= 1e-5 normwise, principal angles <= 1e-4 rad on
the gap-separated scope, and U, V orthonormal to 1e-5.  ``sweeps`` tells the
two core paths apart: the secular path reports 0."""
import numpy as np
import pytest

from oracle.engine import OracleEngine
from synth.factor_model import ROW, COL
from tests.parity import compare

pytestmark = pytest.mark.gpu

M0, N0, K = 120, 40, 8


@pytest.fixture(scope="module")
def isvd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_24514_amd import isvd as mod
    return mod


class _Ev:
    def __init__(self, kind, vec):
        self.kind, self.vec = kind, vec


def _orthonormal(rng, rows, cols):
    q, _ = np.linalg.qr(rng.standard_normal((rows, cols)))
    return q


def _coordinate(rows, idx):
    B = np.zeros((rows, len(idx)))
    B[idx, np.arange(len(idx))] = 1.0
    return B


def _run(isvd, U, S, V, events):
    A0 = (U * S) @ V.T
    o = OracleEngine.from_state(A0, U, S, V, tol_rel=1e-5, cgs2=True)
    sweeps = []
    with isvd.Engine() as eng:
        sid = eng.init_from_factors(A0, U, S, V, "fp32", m_cap=M0 + len(events), n_cap=N0 + len(events),
                                    tol_rel=1e-5)
        for ev in events:
            if ev.kind == ROW:
                eng.append_row(sid, ev.vec)
            else:
                eng.append_col(sid, ev.vec)
            o.apply(ev)
            met = eng.metrics(sid)
            sweeps.append(met["sweeps"])
            Ug, Sg, Vg = eng.factors(sid)
            c = compare((Ug, Sg, Vg), (o.U, o.s, o.V))
            assert c["recon"] <= 2e-5, (ev.kind, c)
            assert c["sigma"] <= 1e-5, (ev.kind, c)
            assert c["angle_U"] <= 1e-4 and c["angle_V"] <= 1e-4, (ev.kind, c)
            kg = len(Sg)
            assert np.abs(Ug.T @ Ug - np.eye(kg)).max() <= 1e-5
            assert np.abs(Vg.T @ Vg - np.eye(kg)).max() <= 1e-5
            assert met["k"] == len(o.s)
    return sweeps


def test_generic_appends_take_the_secular_path(isvd):
    rng = np.random.default_rng(11)
    U, V = _orthonormal(rng, M0, K), _orthonormal(rng, N0, K)
    S = np.array([9.0, 7.5, 6.1, 4.0, 3.3, 2.0, 1.2, 0.7])
    events = []
    for t in range(6):
        if t % 2 == 0:
            events.append(_Ev(ROW, rng.standard_normal(N0 + t // 2)))
        else:
            events.append(_Ev(COL, rng.standard_normal(M0 + (t + 1) // 2)))
    sweeps = _run(isvd, U, S, V, events)
    assert all(s == 0 for s in sweeps), sweeps


def test_repeated_singular_values_merge_poles(isvd):
    rng = np.random.default_rng(12)
    U, V = _orthonormal(rng, M0, K), _orthonormal(rng, N0, K)
    S = np.array([4.0, 4.0, 4.0, 2.0, 2.0, 1.0, 1.0, 1.0])
    events = [_Ev(ROW, rng.standard_normal(N0)), _Ev(COL, rng.standard_normal(M0 + 1)),
              _Ev(ROW, 0.5 * rng.standard_normal(N0 + 1))]
    sweeps = _run(isvd, U, S, V, events)
    assert sweeps[0] == 0 and sweeps[1] == 0, sweeps


def test_zero_weights_deflate(isvd):
    """Coordinate bases: a row along one right vector (one nonzero weight, no
    new direction), a row orthogonal to V (rho the only weight), then the
    same two cases for columns against U."""
    U = _coordinate(M0, [3, 10, 17, 25, 40, 51, 77, 90])
    V = _coordinate(N0, [0, 2, 5, 9, 14, 20, 27, 33])
    S = np.array([8.0, 6.0, 5.0, 3.5, 3.0, 2.0, 1.5, 1.0])
    x1 = np.zeros(N0)
    x1[5] = 3.0
    x2 = np.zeros(N0)
    x2[11] = 2.5
    y1 = np.zeros(M0 + 2)
    y1[10] = -4.0
    y2 = np.zeros(M0 + 2)
    y2[60] = 1.75
    events = [_Ev(ROW, x1), _Ev(ROW, x2), _Ev(COL, y1), _Ev(COL, y2)]
    sweeps = _run(isvd, U, S, V, events)
    assert all(s == 0 for s in sweeps), sweeps


def test_wide_spectrum_falls_back_to_jacobi(isvd):
    rng = np.random.default_rng(13)
    U, V = _orthonormal(rng, M0, K), _orthonormal(rng, N0, K)
    S = np.array([1e3, 10.0, 1.0, 0.5, 0.2, 0.1, 0.05, 0.01])
    events = [_Ev(ROW, 0.01 * rng.standard_normal(N0)), _Ev(COL, 0.01 * rng.standard_normal(M0 + 1))]
    sweeps = _run(isvd, U, S, V, events)
    assert all(s > 0 for s in sweeps), sweeps
