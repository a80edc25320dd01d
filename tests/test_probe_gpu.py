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


def test_hbm_probe_copies_and_stays_under_the_peak():
    from paper_2507_01152_amd import sonosim as sg
    from paper_2507_01152_amd.session import Session
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with Session(0) as s:
        src = torch.arange(1 << 26, dtype=torch.int32, device=s.device)    # 256 MiB
        dst = torch.zeros_like(src)
        rate = sg.sg_hbm_probe(s.ctx, src, dst)
        torch.cuda.synchronize()
        assert torch.equal(src, dst)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        dst.copy_(src)
        ev0.record()
        for _ in range(3):
            dst.copy_(src)
        ev1.record()
        torch.cuda.synchronize()
        t_gbs = 3 * 2 * src.numel() * 4 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
        print(f"device copy {rate / 1e9:.0f} GB/s (read + written); torch copy_ {t_gbs:.0f} GB/s")
        assert 0.3 * 8e12 < rate <= 1.02 * 8e12
        # a ragged tail: 16-byte multiples that are not multiples of the grid
        a = torch.arange(1000004, dtype=torch.int32, device=s.device)
        b = torch.zeros_like(a)
        sg.sg_hbm_probe(s.ctx, a, b)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        # sizes that are not multiples of 16 bytes and overlapping buffers are refused on the host
        odd = torch.zeros(3, dtype=torch.int32, device=s.device)
        with pytest.raises(sg.SonosimError):
            sg.sg_hbm_probe(s.ctx, odd, torch.zeros_like(odd))
        with pytest.raises(sg.SonosimError):
            sg.sg_hbm_probe(s.ctx, a[:8], a[4:12])
