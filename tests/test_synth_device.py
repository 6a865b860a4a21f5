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


@pytest.mark.gpu
def test_async_rows_match_the_synchronous_generator():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from synth import device
    st = torch.cuda.Stream()
    gen = device.AsyncRows(300, 90, 5)
    # two panels in a row on one stream (the second smaller), the buffers reused in stream order
    for (row0, rows, cols, s) in [(0, 300, 90, 4), (77, 41, 33, 9)]:
        ref = torch.empty((rows, cols), dtype=torch.float32, device="cuda")
        device.rows_into(ref, row0, rows, cols, 3, s, 5)
        with torch.cuda.stream(st):
            got = torch.empty((rows, cols), dtype=torch.float32, device="cuda")
            gen.rows_into(got, row0, rows, cols, 3, s, st.cuda_stream)
        st.synchronize()
        assert torch.equal(got, ref)
    with pytest.raises(ValueError):
        gen.rows_into(ref, 0, 301, 10, 3, 0, st.cuda_stream)
