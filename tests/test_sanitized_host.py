"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer: the
FP64 oracle (plain C) and the HIP library's host side (argument validation,
packing, batch layout, workspace checks; the device code is built as usual)
are rebuilt with the sanitizers into a temporary directory, and the rest of
the CPU suite runs against those builds in a child process with the
sanitizer runtime preloaded.  Any report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    out = subprocess.run(["/opt/rocm/llvm/bin/clang", "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_cpu_suite_under_sanitizers(tmp_path):
    rt = _asan_runtime()
    if rt is None or not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("clang sanitizer runtime or hipcc not available")
    sys.path.insert(0, ROOT)
    from oracle import build_oracle
    from paper_2102_01747_amd import _build

    olib = build_oracle.build(sanitize=True, out=str(tmp_path / "liboracle_san.so"))
    flib = _build.build(sanitize=True, out=str(tmp_path / "libfrt_san.so"))
    env = dict(os.environ)
    env.update({"LD_PRELOAD": rt, "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
                "FRT_LIB_PATH": flib, "FRT_ORACLE_LIB": olib, "OMP_NUM_THREADS": "4"})
    probe = ("import sys; sys.path.insert(0, %r); import paper_2102_01747_amd as f; from oracle import oracle as o; "
             "f.lib(); o.lib(); print(open('/proc/self/maps').read())" % ROOT)
    maps = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=300).stdout
    assert flib in maps and olib in maps and "libclang_rt.asan" in maps
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
           "--ignore", os.path.join(ROOT, "tests", "test_sanitized_host.py"), os.path.join(ROOT, "tests")]
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    log = res.stdout + res.stderr
    print(log[-3000:])
    assert res.returncode == 0, log[-6000:]
    for marker in ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer"):
        assert marker not in log, log[-6000:]
    # the child really ran against the sanitised builds
    assert " passed" in log
