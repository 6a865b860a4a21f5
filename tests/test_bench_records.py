"""Host logic of bench.py's roofline report: the committed counter records
parse, their traffic ratios are plausible, and a record whose kernel sources
no longer hash to the profiled ones is ignored (the bench then reports no
traffic rather than a stale one)."""
import os
import re

import bench


def _keys(path):
    out = {}
    for line in open(path).read().splitlines():
        m = re.match(r"^([a-z_0-9]+): *(\S+)$", line)
        if m:
            out[m.group(1)] = m.group(2)
    return out


def test_records_parse():
    for (path, sources), keys in ((bench.PMC_ROTATE, ["traffic_over_algorithmic_variant_%d" % v for v in range(5)]),
                                  (bench.PMC_CORE, ["traffic_over_algorithmic"])):
        kv = _keys(path)
        assert re.fullmatch(r"[0-9a-f]{64}", kv["kernel_source_sha256"])
        for key in keys:
            assert 1.0 <= float(kv[key]) <= 1.5, (path, key)
        assert all(os.path.exists(f) for f in sources)


def test_stale_record_is_ignored(tmp_path):
    path, sources = bench.PMC_CORE
    text = open(path).read()
    ok = bench.recorded_traffic_ratio((path, sources), "traffic_over_algorithmic")
    bad = tmp_path / "rec.md"
    bad.write_text(re.sub(r"kernel_source_sha256: *[0-9a-f]+", "kernel_source_sha256: " + "0" * 64, text))
    assert bench.recorded_traffic_ratio((str(bad), sources), "traffic_over_algorithmic") is None
    if ok is not None:
        assert ok == float(_keys(path)["traffic_over_algorithmic"])
    assert bench.recorded_traffic_ratio((str(tmp_path / "missing.md"), sources), "traffic_over_algorithmic") is None


def test_byte_models():
    assert bench.core_bytes(64) == 32 * 64 * 64 + 4 * 64 * 65
    # deferred U moves U's pass to one append in m / (8 k)
    m, n, k = 40000, 1000, 64
    full = bench.tick_bytes(m, n, k, 4)
    dfr = bench.tick_bytes(m, n, k, 4, deferred=True)
    period = m // (8 * k)
    assert abs((full - dfr) - bench.rot_u_bytes(m, k, 4) * (1 - 1 / period)) <= 1e-6 * full
