"""The device generator reproduces the host generator's panel entries."""
import numpy as np
import pytest

from synth import FactorStream


@pytest.mark.gpu
def test_device_rows_match_host_generator():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from synth import device
    fs = FactorStream(seed=3, stream=17, n0=75, K=5)
    host = fs.initial(130)
    out = torch.empty((130, 75), dtype=torch.float64, device="cuda")
    device.rows_into(out, 0, 130, 75, 3, 17, 5)
    dev = out.cpu().numpy()
    # identical up to the last bits of log / sin / cos
    assert np.max(np.abs(dev - host)) <= 1e-13 * np.max(np.abs(host))
    # appended rows at any offset, float32 storage
    out32 = torch.empty((4, 75), dtype=torch.float32, device="cuda")
    device.rows_into(out32, 1000, 4, 75, 3, 17, 5)
    for r in range(4):
        ref = fs.row(1000 + r, 75).astype(np.float32)
        got = out32[r].cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 2 * np.finfo(np.float32).eps * np.max(np.abs(ref))
