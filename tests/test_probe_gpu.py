"""The VALU throughput probe behind the ALU roofline's peak (GPU)."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz: the FP32 vector peak (157.3 TFLOP/s) in lane-ops/s
PEAK = 256 * 4 * 32 * 2.4e9


def test_valu_probe_rates_bound_the_roofline():
    from paper_2507_01152_amd import sonosim as sg
    from paper_2507_01152_amd.session import Session
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with Session(0) as s:
        fma2, xa, mad, fma3 = sg.sg_valu_probe(s.ctx)
    print(f"FMA (2-operand) {fma2 / 1e12:.1f}, xor/add {xa / 1e12:.1f}, mad_u64 {mad / 1e12:.1f}, "
          f"FMA (3-operand) {fma3 / 1e12:.1f} T lane-ops/s")
    # the derived peak bounds what independent chains reach, and two-operand chains reach most of it
    for r in (fma2, xa):
        assert 0.5 * PEAK < r <= 1.02 * PEAK
    assert fma3 <= fma2
    # the 32x32->64 multiply-add issues at a fraction of the simple-op rate (weighted 4 in the op count)
    assert mad < 0.5 * xa
