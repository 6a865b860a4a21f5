"""Full-size single stream (the 100000 x 2000 panel with 20 factors, k = 64):
the GPU's FP64 and FP32 update paths against the FP64 oracle's Brand updates
from the same starting factors, over a mixed run of row appends, column
appends and rank-1 entry updates (80/10/10), plus properties that hold at
any size: orthonormal bases, the tracked ||A||^2 against a direct sum, and
E_inc from the GPU's residual pass against a blockwise host evaluation.

The starting factors are the GPU FP64 engine's TruncatedSVD of A_0 (the
oracle's own Jacobi SVD of a 100000 x 2000 panel would take minutes); the
oracle then runs Alg. A1-A3 on them directly (it needs no A for that)."""
import numpy as np
import pytest

from synth import FactorStream, event_schedule_iid, ROW, COL, ENTRY
from oracle import brand
from tests.parity import compare

pytestmark = pytest.mark.gpu

M0, N0, K, NF, T = 100000, 2000, 64, 20, 16


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_24514_amd import isvd
    from synth import device as sdev
    return torch, isvd, sdev


def _oracle_apply(U, s, V, ev, tol_rel):
    if ev.kind == ROW:
        U, s, V, _ = brand.row_append(U, s, V, ev.vec, K, tol_rel, cgs2=True)
    elif ev.kind == COL:
        U, s, V, _ = brand.col_append(U, s, V, ev.vec, K, tol_rel, cgs2=True)
    else:
        U, s, V = brand.rank_one(U, s, V, ev.i, ev.j, ev.delta)
    return U, s, V


def test_large_stream_mixed_updates_match_the_oracle(env):
    torch, isvd, sdev = env
    fs = FactorStream(seed=21, stream=0, n0=N0, K=NF)
    kinds = event_schedule_iid(21, 0, T, mix=(0.8, 0.1, 0.1))
    kinds = [ROW, COL, ENTRY] + list(kinds[3:])          # every kind at least once
    events = fs.materialize(kinds, m0=M0)
    A0 = torch.empty((M0, N0), dtype=torch.float64, device="cuda")
    sdev.rows_into(A0, 0, M0, N0, 21, 0, NF)
    with isvd.Engine() as e64, isvd.Engine() as e32:
        s64 = e64.init(A0, K, "fp64", m_cap=M0 + T, n_cap=N0 + T, refresh_iters=2)
        U, S, V = e64.factors(s64)
        s32 = e32.init_from_factors(A0, U, S, V, "fp32", m_cap=M0 + T, n_cap=N0 + T)
        oU, os_, oV = U.copy(), S.copy(), V.copy()
        o32 = (U.copy(), S.copy(), V.copy())
        for ev in events:
            for eng, sid in ((e64, s64), (e32, s32)):
                if ev.kind == ROW:
                    eng.append_row(sid, ev.vec)
                elif ev.kind == COL:
                    eng.append_col(sid, ev.vec)
                else:
                    eng.update_entry(sid, ev.i, ev.j, ev.delta)
            oU, os_, oV = _oracle_apply(oU, os_, oV, ev, 1e-10)
            o32 = _oracle_apply(*o32, ev, 1e-5)
        c64 = compare(e64.factors(s64), (oU, os_, oV))
        c32 = compare(e32.factors(s32), o32)
        print("fp64", c64)
        print("fp32", c32)
        assert c64["recon"] <= 1e-10 and c64["sigma"] <= 1e-12, c64
        assert c32["recon"] <= 2e-5 and c32["sigma"] <= 1e-5, c32
        assert c32["angle_U"] <= 1e-4 and c32["angle_V"] <= 1e-4, c32
        # properties at full size (FP32 engine): orthonormality, N_t, E_inc
        met = e32.metrics(s32, exact=True)
        assert met["ortho_U"] <= 1e-5 and met["ortho_V"] <= 1e-5, met
        A = e32.matrix(s32)
        fro2 = float(np.sum(A * A))
        assert abs(met["fro2_A"] - fro2) <= 1e-6 * fro2
        Ug, Sg, Vg = e32.factors(s32)
        SVt = (Vg * Sg).T
        r2 = 0.0
        for r0 in range(0, A.shape[0], 20000):
            D = A[r0:r0 + 20000] - Ug[r0:r0 + 20000] @ SVt
            r2 += float(np.sum(D * D))
        assert abs(met["frob_error"] - np.sqrt(r2)) <= 1e-6 * np.sqrt(fro2), (met["frob_error"], np.sqrt(r2))
        assert met["frob_error"] >= met["frob_opt"] * (1 - 1e-6)
