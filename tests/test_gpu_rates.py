"""The vector-unit rate probes: sustained FP32 FMA and hardware
transcendental rates over the whole device, the ceilings the march kernels
are measured against.  With packed FP32 instructions off, one FMA per lane
per cycle on 256 compute units of four 16-lane SIMDs at up to 2.4 GHz is
78.6 TFLOP/s; the transcendentals issue at a quarter of the FMA rate or
less.  The mix probe shows whether transcendentals overlap FMAs."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frt():
    import paper_2102_01747_amd as m
    m.lib()
    return m


def test_fma_rate_near_the_nonpacked_ceiling(frt):
    tflops = frt.valu_rate("fma", 16384) * 2 / 1e12
    print("FP32 FMA: %.1f TFLOP/s" % tflops)
    # below the non-packed ceiling at the top clock, and not far below it
    assert 0.5 * 78.6 < tflops < 1.02 * 78.6


@pytest.mark.parametrize("op", ["exp2", "log2", "rsq", "rcp", "sqrt", "sin_rev"])
def test_transcendental_rates(frt, op):
    fma = frt.valu_rate("fma", 16384)
    r = frt.valu_rate(op, 4096)
    print("%s: %.2f T lane-ops/s, %.3f of the FMA rate" % (op, r / 1e12, r / fma))
    assert 0.05 * fma < r < 1.05 * fma


def test_mix_of_fma_and_exp2(frt):
    fma = frt.valu_rate("fma", 16384)
    ex = frt.valu_rate("exp2", 4096)
    mix = frt.valu_rate("fma4_exp2", 4096)
    # time per chain round if the 4 FMAs and the exp2 issue one after another
    serial = 4 / fma + 1 / ex
    overlap = max(4 / fma, 1 / ex)
    measured = 5 / mix
    print("4 FMA + exp2 per round: measured %.3e s, serial %.3e, fully overlapped %.3e (lane-round)"
          % (measured, serial, overlap))
    assert 0.8 * overlap < measured < 1.25 * serial



@pytest.mark.parametrize("op", ["fadd", "fmul", "int_shift_add"])
def test_other_vector_op_rates(frt, op):
    """FP32 add and multiply, and integer shift-and-add chains: the issue
    rate of the non-FMA instructions that make up the rest of the march
    kernels' vector work, against the FMA rate."""
    fma = frt.valu_rate("fma", 16384)
    r = frt.valu_rate(op, 8192)
    print("%s: %.2f T lane-ops/s, %.3f of the FMA rate" % (op, r / 1e12, r / fma))
    assert 0.3 * fma < r < 4.0 * fma
