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
    assert L.frt_valu_rate(11, 16, ctypes.byref(r), None) == frt.FRT_EINVAL
    assert L.frt_valu_rate(-1, 16, ctypes.byref(r), None) == frt.FRT_EINVAL
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


def test_render_validation_on_the_host():
    """Every check of a render's parameters and workspace runs before the
    library touches a device, so each invalid case is host-testable: exact
    status code and a message naming the field.  The output pointers are
    fake and never dereferenced."""
    import copy

    import paper_2102_01747_amd as frt
    import workloads as W

    if not os.path.exists(frt.LIB_PATH):
        pytest.skip("libfrt.so not built")
    L = frt.lib()
    fake = ctypes.c_void_p(0x10000)
    out = frt.Frame(fake, fake, fake, fake, None)
    ws = ctypes.c_void_p(0x100000)   # 256-byte aligned, never dereferenced
    base = W.julia_view(width=16, height=16, planes=[W.plane([0.0, 0.0, 1.0], 0.1)])

    def call(job, frame=out, workspace=ws, ws_bytes=1 << 20, n_planes=None):
        planes, npl = frt.make_planes(job["planes"])
        return L.frt_render(ctypes.byref(frt.make_camera(job["camera"])), ctypes.byref(frt.make_fractal(job["fractal"])),
                            planes, npl if n_planes is None else n_planes, ctypes.byref(frt.make_march(job["march"])),
                            frame, workspace, ws_bytes, None)

    def case(edit, status, words, **kw):
        job = copy.deepcopy(base)
        edit(job)
        assert call(job, **kw) == status, words
        assert words.encode() in L.frt_last_error(), (words, L.frt_last_error())

    def setitem(path, value):
        def f(job):
            d = job
            for k in path[:-1]:
                d = d[k]
            d[path[-1]] = value
        return f

    case(setitem(("camera", "width"), 0), frt.FRT_EINVAL, "width and height")
    case(setitem(("camera", "fov_y_deg"), 180.0), frt.FRT_EINVAL, "fov_y_deg")
    case(setitem(("fractal", "c"), [float("nan"), 0.0, 0.0, 0.0]), frt.FRT_EINVAL, "non-finite fractal")
    case(setitem(("fractal", "kind"), 7), frt.FRT_EINVAL, "unknown fractal kind")
    case(setitem(("fractal", "power"), 17.0), frt.FRT_EINVAL, "Julia degree")
    case(setitem(("fractal", "max_iter"), 0), frt.FRT_EINVAL, "max_iter")
    case(setitem(("planes",), [W.plane([0.0, 0.0, 0.0], 0.1)]), frt.FRT_EINVAL, "plane normal is zero")
    case(lambda j: None, frt.FRT_EINVAL, "n_planes", n_planes=3)
    case(lambda j: j["march"].update(eps_abs=0.0, eps_rel=0.0), frt.FRT_EINVAL, "eps_abs and eps_rel")
    case(setitem(("march", "step_clamp"), 0.0), frt.FRT_EINVAL, "step_clamp")
    case(setitem(("march", "normal_mode"), 5), frt.FRT_EINVAL, "unknown normal_mode")
    case(setitem(("march", "refine_iters"), 33), frt.FRT_EINVAL, "refine_iters")
    case(lambda j: None, frt.FRT_EINVAL, "null output plane", frame=frt.Frame(fake, None, fake, fake, None))
    # the closest-hit model: its palette is validated like every parameter
    bad_pal = [[0.0] * 3, [float("inf"), 0.0, 0.0], [0.0] * 3, [0.0] * 3]
    case(lambda j: j.update(march=dict(W.phong(j["march"]), trap_colour=bad_pal)), frt.FRT_EINVAL, "trap_colour")
    # a valid job, then the workspace checks
    case(lambda j: None, frt.FRT_EINVAL, "workspace is null", workspace=None)
    case(lambda j: None, frt.FRT_EINVAL, "aligned", workspace=ctypes.c_void_p(0x100008))
    case(lambda j: None, frt.FRT_ENOMEM, "workspace too small", ws_bytes=64)


def test_batch_and_backward_validation_on_the_host():
    """frt_render_batch names the first invalid job; frt_render_backward
    refuses analytic normals and the closest-hit shading: all before any
    device call (fake, never dereferenced pointers)."""
    import copy

    import paper_2102_01747_amd as frt
    import workloads as W

    if not os.path.exists(frt.LIB_PATH):
        pytest.skip("libfrt.so not built")
    L = frt.lib()
    fake = ctypes.c_void_p(0x10000)
    ws = ctypes.c_void_p(0x100000)
    good = W.julia_view(width=16, height=16)
    bad = copy.deepcopy(good)
    bad["fractal"]["max_iter"] = 0

    def table(jobs):
        arr = (frt.Job * len(jobs))()
        for k, j in enumerate(jobs):
            planes, npl = frt.make_planes(j["planes"])
            arr[k] = frt.Job(frt.make_camera(j["camera"]), frt.make_fractal(j["fractal"]), planes, npl,
                             frt.make_march(j["march"]), frt.Frame(fake, fake, fake, fake, None))
        return arr

    arr = table([good, good, bad])
    assert L.frt_render_batch(arr, 3, ws, 1 << 20, 0, None) == frt.FRT_EINVAL
    assert b"job 2" in L.frt_last_error() and b"max_iter" in L.frt_last_error()
    assert L.frt_render_batch(table([good]), 1, ws, 1 << 20, 2, None) == frt.FRT_EINVAL   # use_graph
    assert L.frt_render_batch(table([good]), 1, ws, 64, 0, None) == frt.FRT_ENOMEM
    # the entry point that allocates nothing checks the same before any device
    # call, and leaves the closest-hit model to the other renderers
    phong1 = copy.deepcopy(good)
    phong1["march"] = W.phong(phong1["march"])
    assert L.frt_render_batch_noalloc(table([good, phong1]), 2, None) == frt.FRT_EUNSUPPORTED
    assert b"job 1" in L.frt_last_error()
    assert L.frt_render_batch_noalloc(arr, 3, None) == frt.FRT_EINVAL
    assert b"job 2" in L.frt_last_error() and b"max_iter" in L.frt_last_error()
    assert L.frt_render_batch_noalloc(None, 1, None) == frt.FRT_EINVAL
    assert L.frt_render_batch_noalloc(table([good]), 0, None) == frt.FRT_EINVAL
    big = table([good] * (frt.NOALLOC_MAX_JOBS + 1))
    assert L.frt_render_batch_noalloc(big, frt.NOALLOC_MAX_JOBS + 1, None) == frt.FRT_EINVAL
    assert b"FRT_NOALLOC_MAX_JOBS" in L.frt_last_error()
    assert frt.noalloc_scratch_bytes() == frt.workspace_bytes(frt.NOALLOC_MAX_JOBS) <= 256 << 10

    analytic = copy.deepcopy(good)
    analytic["march"]["normal_mode"] = "analytic"
    g = ctypes.c_void_p(0x200000)
    assert L.frt_render_backward(table([good, analytic]), 2, None, None, None, None, g, g, g, ws, 1 << 20,
                                 None) == frt.FRT_EUNSUPPORTED
    assert b"job 1" in L.frt_last_error() and b"second derivatives" in L.frt_last_error()
    phong = copy.deepcopy(good)
    phong["march"] = W.phong(phong["march"])
    assert L.frt_render_backward(table([phong]), 1, None, None, None, None, g, g, g, ws, 1 << 20,
                                 None) == frt.FRT_EUNSUPPORTED
    assert L.frt_render_backward(table([good]), 1, None, None, None, None, None, g, g, ws, 1 << 20,
                                 None) == frt.FRT_EINVAL
