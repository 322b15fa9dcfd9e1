"""Build the HIP library libfrt.so for gfx950 in-tree.

One hipcc link of the kernel translation units and the host API.  Every HIP
source is compiled with packed-FP32 instructions disabled
(-target-feature -packed-fp32-ops): the kernels are written for plain
single-lane FP32 issue.  Sources listed in SOURCE_FLAGS are first compiled to
objects of their own with those flags added.
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

# The forward kernels run with FP32 denormals flushed and the hardware's IEEE
# mode off, with no NaN and no signed-zero semantics: the orbit bodies then
# double a product through the multiply's output modifier instead of a
# separate add (omod, which the hardware honours only in that mode).  Their
# values never reach the denormal range, NaN or a signed zero on any path the
# outputs depend on.  The FP64 adjoint and the other kernels keep strict IEEE
# semantics.
FORWARD_FP_MODE = ["-fgpu-flush-denormals-to-zero", "-mno-amdgpu-ieee", "-fno-honor-nans", "-fno-signed-zeros"]
SOURCE_FLAGS = {"frt_trace.hip": FORWARD_FP_MODE}


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

# The strict build: the same sources with no per-source flags, every kernel
# in strict IEEE semantics; the tests require the forward kernels' outputs to
# equal the product build's bit for bit.
STRICT_LIB = os.path.join(PKG, "libfrt_strict.so")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if verbose and out.strip():
        print(out, flush=True)


def build(verbose: bool = False, sanitize: bool = False, out: str = None, instrument: bool = False,
          csrc: str = None, source_flags: dict = None, strict: bool = False) -> str:
    csrc = csrc or CSRC
    source_flags = ({} if strict else SOURCE_FLAGS) if source_flags is None else source_flags
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(csrc, s))]
    dest = out or (INSTR_LIB if instrument else STRICT_LIB if strict else LIB)
    tmp = dest + ".tmp"
    opt = SANITIZE_HOST.split() if sanitize else ["-O3"]
    if instrument:
        opt = opt + ["-DFRT_TRIP_COUNTERS", "-DFRT_DEBUG_CHECKS"]
    common = [hipcc(), "--offload-arch=" + ARCH] + opt + ["-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Wall", "-I", INCLUDE, "-I", csrc]
    inputs, objs = [], []
    for s in srcs:
        path = os.path.join(csrc, s)
        if source_flags.get(s):
            obj = "%s.%s.o" % (tmp, s)
            _run(common + source_flags[s] + ["-c", path, "-o", obj], verbose)
            objs.append(obj)
            inputs.append(obj)
        else:
            inputs.append(path)
    try:
        _run(common + ["-shared"] + inputs + ["-o", tmp], verbose)
    finally:
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)
    os.replace(tmp, dest)
    return dest


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
