"""Input generator: Philox known answers, normal statistics, factor-model consistency."""
import os

import numpy as np
import pytest

from synth import philox4x32_10, normals, uniforms, FactorStream, factor_lambdas
from synth import event_schedule_c0, event_schedule_iid, ROW, COL, ENTRY

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        vals = [int(v, 16) for v in r]
        out = philox4x32_10(*vals[:6])
        assert [int(o) for o in out] == vals[6:]


def test_normals_statistics_and_prefix():
    z = normals(7, 3, 2, np.arange(64), 1000)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
    # a longer draw extends a shorter one (each entry has its own counter)
    z2 = normals(7, 3, 2, np.arange(64), 1001)
    assert np.array_equal(z2[:, :1000], z)
    u = uniforms(7, 3, 2, np.arange(8), 10000)
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.01
    # distinct purposes / streams / seeds give distinct draws
    assert not np.allclose(normals(7, 3, 3, [0], 8), normals(7, 3, 2, [0], 8))
    assert not np.allclose(normals(7, 4, 2, [0], 8), normals(7, 3, 2, [0], 8))


def test_lambdas_reproduce_five_factor_variances():
    assert np.allclose(factor_lambdas(5), [4, 2, 1, 0.5, 0.25])
    lam = factor_lambdas(20)
    assert lam[0] == 4.0 and abs(lam[-1] - 0.25) < 1e-15 and np.all(np.diff(lam) < 0)


def test_factor_stream_rows_and_columns_are_consistent():
    fs = FactorStream(seed=0, stream=0, n0=50, K=5)
    A = fs.initial(40)
    # row i of the initial panel is what a row append at index i would emit
    assert np.array_equal(fs.row(17, 50), A[17])
    # an appended column uses the stored factors of every existing row
    y = fs.col(50, 40)
    F = fs.factors(0, 40)
    b = fs.loadings(50, 51)[0]
    resid = y - F @ b
    assert np.std(resid) < 0.15 and np.std(resid) > 0.05
    # the model is rank-5 plus 0.1 noise
    s = np.linalg.svd(A, compute_uv=False)
    assert s[4] > 10 * s[5]


def test_event_schedules():
    kinds = event_schedule_c0(0, 0, 1000, 200)
    assert kinds.count(ROW) == 1000 and kinds.count(ENTRY) == 200
    kinds2 = event_schedule_iid(1, 0, 20000, (0.8, 0.1, 0.1))
    frac = np.bincount(kinds2, minlength=3) / 20000.0
    assert np.allclose(frac, [0.8, 0.1, 0.1], atol=0.01)


def test_materialize_tracks_shapes():
    fs = FactorStream(seed=1, stream=2, n0=30, K=5)
    evs = fs.materialize([ROW, COL, ENTRY, ROW], m0=20)
    assert evs[0].vec.shape == (30,)
    assert evs[1].vec.shape == (21,)
    assert 0 <= evs[2].i < 21 and 0 <= evs[2].j < 31
    assert evs[3].vec.shape == (31,)
    assert [e.t for e in evs] == [1, 2, 3, 4]


def test_device_generator_rejects_outputs_it_cannot_fill():
    """The device generator's host checks turn an output that is not a
    contiguous device tensor of the right size into an error before any
    launch (checked here on the CPU, where no launch can happen)."""
    torch = pytest.importorskip("torch")
    from synth import device
    with pytest.raises(ValueError):
        device.rows_into(torch.empty((4, 5), dtype=torch.float32), 0, 4, 5, 1, 0, 3)
    with pytest.raises(TypeError):
        device.rows_into(torch.empty((4, 5), dtype=torch.int32), 0, 4, 5, 1, 0, 3)
