"""Checks on the compiled device code of the march kernels (no GPU needed).

The ROCm 7.2 compiler was seen to compile one form of the march kernels'
claim loop so that an s_cselect read the scalar condition flag left by a
64-bit address add (its carry) instead of the 64-bit bound test just made on
the vector unit; the shadow march then stopped after its second chunk of
rays.  The test compiles frt_trace.hip to gfx950 assembly with the library's
own flags and fails if any select or conditional scalar move reads a condition
flag last written by an add, subtract or shift with a vector compare in
between -- the shape of that miscompile.

The same assembly must hold no function calls: the forward kernels are built
in another floating-point mode than the device library's, and a library
function reached from them (HIP's thread-index accessors, rsqrtf) is then not
inlined but called, with the call's register convention around it.
"""
import os
import re
import subprocess

import pytest

from paper_2102_01747_amd import _build

# scalar instructions that leave the condition flag alone
_KEEP = ("s_mov", "s_cmov", "s_cselect", "s_mul_i32", "s_mul_hi", "s_load", "s_store", "s_buffer", "s_waitcnt",
         "s_nop", "s_branch", "s_cbranch", "s_getpc", "s_setpc", "s_swappc", "s_endpgm", "s_memrealtime",
         "s_memtime", "s_barrier", "s_sleep", "s_setprio", "s_sext", "s_brev", "s_bitset", "s_movk", "s_getreg",
         "s_setreg", "s_sendmsg", "s_dcache", "s_icache", "s_trap", "s_pack", "s_set_gpr", "s_denorm", "s_round",
         "s_inst_prefetch", "s_delay", "s_wait")
_ARITH = re.compile(r"^s_(add|addc|sub|subb|lshl|lshr|ashr)")


def stale_flag_selects(asm_text):
    """(kernel, line, instruction) of every s_cselect / s_cmov reading a flag
    written by arithmetic with a vector compare issued since."""
    out = []
    kern, last, vcmp = None, None, False
    for i, line in enumerate(asm_text.splitlines()):
        m = re.match(r"^(_Z\S+):", line)
        if m:
            kern, last, vcmp = m.group(1), None, False
            continue
        tok = line.strip().split()
        if not tok or tok[0].startswith((";", ".")):
            continue
        op = tok[0]
        if op.startswith("v_cmp"):
            vcmp = True
        if op.startswith(("s_cselect", "s_cmov")) and last and _ARITH.match(last) and vcmp:
            out.append((kern, i + 1, line.strip()))
        if op.startswith("s_") and not op.startswith(_KEEP):
            last, vcmp = op, False
    return out


def test_detector_flags_the_pattern():
    bad = "_Zk:\n\ts_add_u32 s6, s6, s24\n\ts_addc_u32 s7, s8, s25\n\tv_cmp_lt_u64_e32 vcc, s[6:7], v[6:7]\n" \
          "\ts_cselect_b32 s7, s7, s27\n"
    good = "_Zk:\n\ts_add_u32 s6, s6, s24\n\tv_cmp_lt_u64_e32 vcc, s[6:7], v[6:7]\n\ts_and_b64 s[4:5], vcc, exec\n" \
           "\ts_cselect_b32 s7, s7, s27\n"
    assert len(stale_flag_selects(bad)) == 1
    assert stale_flag_selects(good) == []


@pytest.fixture(scope="module")
def trace_asm(tmp_path_factory):
    """gfx950 assembly of frt_trace.hip, compiled with the library's flags."""
    hipcc = _build.hipcc()
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = os.path.join(_build.CSRC, "frt_trace.hip")
    out = tmp_path_factory.mktemp("asm") / "trace.s"
    cmd = [hipcc, "--offload-arch=" + _build.ARCH, "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops"] + _build.SOURCE_FLAGS.get("frt_trace.hip", []) + [
           "-I", _build.INCLUDE, "-I", _build.CSRC, "--cuda-device-only", "-S", src, "-o", str(out)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    return out.read_text()


@pytest.mark.timeout(600)
def test_march_kernels_have_no_stale_flag_select(trace_asm):
    bad = stale_flag_selects(trace_asm)
    assert not bad, "selects on a stale condition flag: %s" % bad[:5]


@pytest.mark.timeout(600)
def test_forward_kernels_make_no_calls(trace_asm):
    calls = re.findall(r"^\s*s_swappc_b64.*$", trace_asm, flags=re.M)
    callees = sorted(set(re.findall(r"(\w+)@rel32@lo", trace_asm)))
    assert not calls, "calls in the forward kernels (%d), to %s" % (len(calls), callees)
