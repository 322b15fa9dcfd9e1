"""Build the HIP library libfrt.so for gfx950 in-tree.

One hipcc link of the kernel translation units and the host API.  Every HIP
source is compiled with packed-FP32 instructions disabled
(-target-feature -packed-fp32-ops): the kernels are written for plain
single-lane FP32 issue.
"""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libfrt.so")
SOURCES = ["frt_trace.hip", "frt_query.hip", "frt_adjoint.hip", "frt_scene.hip", "frt_rates.hip", "frt_noalloc.hip",
           "frt_api.cpp"]
ARCH = os.environ.get("FRT_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer for the CPU
# checks of the host code (argument validation, packing, layout); the device
# code is built as usual.
SANITIZE_HOST = "-O1 -g -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined " \
                "-Xarch_host -fno-sanitize-recover=undefined -Xarch_host -fno-omit-frame-pointer -shared-libsan"


# The instrumented build: the march kernels' trip counters and the kernels'
# index checks (FRT_TRIP_COUNTERS, FRT_DEBUG_CHECKS; see frt_job.hpp); it
# loads like libfrt.so through FRT_LIB_PATH.
INSTR_LIB = os.path.join(PKG, "libfrt_instr.so")


def build(verbose: bool = False, sanitize: bool = False, out: str = None, instrument: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    dest = out or (INSTR_LIB if instrument else LIB)
    tmp = dest + ".tmp"
    opt = SANITIZE_HOST.split() if sanitize else ["-O3"]
    if instrument:
        opt = opt + ["-DFRT_TRIP_COUNTERS", "-DFRT_DEBUG_CHECKS"]
    cmd = [hipcc(), "--offload-arch=" + ARCH] + opt + ["-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-I", INCLUDE, "-I", CSRC] + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if verbose and out.strip():
        print(out, flush=True)
    os.replace(tmp, dest)
    return dest


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
