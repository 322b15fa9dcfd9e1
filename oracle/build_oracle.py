"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

The oracle is plain C99 compiled with gcc, -O2 and no fast-math, so that it
follows IEEE double arithmetic and the C library's libm.

build(sanitize=True, out=...) instead compiles it with clang under
AddressSanitizer and UndefinedBehaviorSanitizer (the LLVM runtime, so that it
can share a process with the host-sanitised HIP library); load it with that
runtime preloaded.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "frt_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
CLANG = "/opt/rocm/llvm/bin/clang"


def build(verbose: bool = False, sanitize: bool = False, out: str = None) -> str:
    out = out or LIB
    tmp = out + ".tmp"
    if sanitize:
        cmd = [CLANG, "-std=gnu99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined", "-shared-libsan", "-fno-fast-math", "-ffp-contract=off",
               "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    else:
        cmd = ["gcc", "-std=gnu99", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
