"""The C ABI library loads and exports every symbol include/isvd.h declares (no GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "isvd.h")).read()
    decl = r"^\s*(?:isvd_status|uint64_t|double|const char\*)\s+(isvd_[a-z_]+)\s*\("
    return sorted(set(re.findall(decl, text, flags=re.M)))


def test_header_declares_the_boundary_calls():
    names = _declared()
    for required in ["isvd_init", "isvd_append_row", "isvd_append_col", "isvd_update_entry",
                     "isvd_refresh", "isvd_metrics", "isvd_tick", "isvd_engine_create"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2605_24514_amd import isvd
    lib = isvd.load_library()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(isvd.EXPORTS) <= set(_declared())


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Sizes and field offsets of the binding's structs equal what gcc lays out."""
    from paper_2605_24514_amd import isvd
    structs = {"isvd_policy": isvd.CPolicy, "isvd_config": isvd.CConfig,
               "isvd_metrics_t": isvd.CMetrics, "isvd_request": isvd.CRequest,
               "isvd_launch_time": isvd.CLaunchTime, "isvd_server_config": isvd.CServerConfig,
               "isvd_completion": isvd.CCompletion, "isvd_server_stats_t": isvd.CServerStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "isvd.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for cname, cls in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got["%s.%s" % (cname, f)]) == getattr(cls, f).offset, (cname, f)


def test_stream_bytes_and_config_validation_without_gpu():
    from paper_2605_24514_amd import isvd
    lib = isvd.load_library()
    cfg = isvd.Engine.config(1000, 50, 10, "fp32", m_cap=2000, n_cap=60)
    b = lib.isvd_stream_bytes(ctypes.byref(cfg))
    # A dominates: 2000 x 60 floats, plus U (3 buffers) and V
    assert b >= 2000 * 60 * 4 + 3 * 2000 * 16 * 4
    bad = isvd.Engine.config(10, 5, 6, "fp32")      # k > min(m0, n0)
    assert lib.isvd_stream_bytes(ctypes.byref(bad)) == 0
    assert b"k = 6" in lib.isvd_last_error()
