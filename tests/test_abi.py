"""The C ABI without a GPU: every function include/frt.h declares is
exported by libfrt.so, and the ctypes structures of the Python binding have
the layout the C compiler gives the header's structs."""
import ctypes
import json
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "frt.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(frt_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("frt_render", "frt_render_batch", "frt_render_backward", "frt_workspace_bytes", "frt_autotune_set",
              "frt_graph_reset", "frt_status_string", "frt_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2102_01747_amd as frt

    if not os.path.exists(frt.LIB_PATH):
        pytest.skip("libfrt.so not built")
    L = ctypes.CDLL(frt.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_host_only_calls_without_gpu():
    """Calls that touch no device: status strings, workspace size, argument
    validation of the tuning table."""
    import paper_2102_01747_amd as frt

    if not os.path.exists(frt.LIB_PATH):
        pytest.skip("libfrt.so not built")
    L = frt.lib()
    assert L.frt_status_string(0) == b"ok"
    assert L.frt_status_string(-1) == b"invalid argument"
    a, b = frt.workspace_bytes(1), frt.workspace_bytes(64)
    assert a % 256 == 0 and b % 256 == 0 and b > a >= 1024
    assert L.frt_autotune_set(99, 64, 256, 0, 8, 16) == frt.FRT_EINVAL
    assert b"kernel_variant" in L.frt_last_error()
    assert L.frt_autotune_set(0, 96, 256, 0, 8, 16) == frt.FRT_EINVAL
    assert L.frt_render_batch(None, 0, None, 0, 0, None) == frt.FRT_EINVAL
    sa, sb = int(L.frt_scene_workspace_bytes(1)), int(L.frt_scene_workspace_bytes(16))
    assert sa % 256 == 0 and sb % 256 == 0 and sb > sa > 1024
    # scene validation happens before anything touches a device
    assert L.frt_render_scene(None, None, 0, None, frt.Frame(), None, None, None, 0, None) == frt.FRT_EINVAL
    assert b"n_objects" in L.frt_last_error()
    # the rate probe checks its arguments before it asks for a device
    r = ctypes.c_double()
    assert L.frt_valu_rate(8, 16, ctypes.byref(r), None) == frt.FRT_EINVAL
    assert L.frt_valu_rate(0, 0, ctypes.byref(r), None) == frt.FRT_EINVAL
    assert L.frt_valu_rate(0, (1 << 20) + 1, ctypes.byref(r), None) == frt.FRT_EINVAL
    assert L.frt_valu_rate(0, 16, None, None) == frt.FRT_EINVAL


def test_ctypes_layout_matches_c_header(tmp_path):
    import paper_2102_01747_amd as frt

    structs = {"frt_camera": frt.Camera, "frt_fractal": frt.Fractal, "frt_plane": frt.Plane,
               "frt_march": frt.March, "frt_frame": frt.Frame, "frt_job": frt.Job, "frt_object": frt.Object}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "frt.h"', "int main(void) {", 'printf("{");']
    first = True
    for cname, py in structs.items():
        for fname, _ in py._fields_:
            sep = "" if first else ","
            first = False
            lines.append('printf("%s\\"%s.%s\\": %%zu", offsetof(%s, %s));' % (sep, cname, fname, cname, fname))
        lines.append('printf(",\\"%s\\": %%zu", sizeof(%s));' % (cname, cname))
    lines += ['printf("}\\n");', "return 0; }"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    got = json.loads(subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout)
    for cname, py in structs.items():
        assert got[cname] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got["%s.%s" % (cname, fname)] == getattr(py, fname).offset, (cname, fname)
