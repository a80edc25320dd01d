"""Pins of the surrogate oracle: torch's bfloat16 conversion, torch FP64
conv2d and its autograd (library routines), central finite differences of
the whole network, and the closed form of a first Adam step.  CPU only."""
import numpy as np
import pytest

from oracle import surrogate as so

torch = pytest.importorskip("torch")
F = torch.nn.functional


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0, 3.0e38])])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(so.bf16_round(x), ref)
    bits = so.f64_to_bf16_bits(x)
    assert np.array_equal(so.bf16_bits_to_f64(bits), ref)


def _torch_conv(x, w, b, stride, pad, up):
    xt = torch.tensor(x).permute(0, 3, 1, 2)
    if up:
        xt = F.interpolate(xt, scale_factor=2, mode="nearest")
    wt = torch.tensor(w).permute(0, 3, 1, 2)
    return F.conv2d(xt, wt, None if b is None else torch.tensor(b), stride=stride, padding=pad)


@pytest.mark.parametrize("k,stride,pad,up", [(3, 1, 1, False), (3, 2, 1, False), (3, 1, 1, True), (1, 1, 0, False),
                                             (3, 2, 0, False)])
def test_conv_ops_match_torch_autograd(k, stride, pad, up):
    rng = np.random.default_rng(1)
    N, H, W, C, Co = 2, 6, 10, 8, 16
    x = rng.standard_normal((N, H, W, C))
    w = rng.standard_normal((Co, k, k, C))
    b = rng.standard_normal(Co)
    y = so.conv_forward(x, w, b, stride=stride, pad=pad, up=up)
    xt = torch.tensor(x, requires_grad=True)
    wt = torch.tensor(w, requires_grad=True)
    bt = torch.tensor(b, requires_grad=True)
    xin = xt.permute(0, 3, 1, 2)
    if up:
        xin = F.interpolate(xin, scale_factor=2, mode="nearest")
    yt = F.conv2d(xin, wt.permute(0, 3, 1, 2), bt, stride=stride, padding=pad).permute(0, 2, 3, 1)
    assert y.shape == tuple(yt.shape)
    assert np.allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    dy = rng.standard_normal(y.shape)
    (yt * torch.tensor(dy)).sum().backward()
    dx = so.conv_backward_data(dy, w, x.shape, stride=stride, pad=pad, up=up)
    dw, db = so.conv_backward_weight(x, dy, k=k, stride=stride, pad=pad, up=up)
    assert np.allclose(dx, xt.grad.numpy(), rtol=1e-12, atol=1e-11)
    assert np.allclose(dw, wt.grad.numpy(), rtol=1e-12, atol=1e-11)
    assert np.allclose(db, bt.grad.numpy(), rtol=1e-12, atol=1e-11)


def _small_problem(seed=3, H=16, W=16):
    rng = np.random.default_rng(seed)
    layout, n = so.param_layout()
    flat = np.zeros(n)
    for name, o, shape in layout:
        fan = int(np.prod(shape[1:])) if name.startswith("w") else 1
        scale = np.sqrt(2.0 / fan) if name.startswith("w") else 0.05
        flat[o:o + int(np.prod(shape))] = rng.standard_normal(int(np.prod(shape))) * scale
    x = np.zeros((1, H, W, 8))
    lab = rng.integers(0, 4, size=(H, W))
    x[0, np.arange(H)[:, None], np.arange(W)[None, :], lab] = 1.0
    x[0, :, :, 4] = rng.standard_normal((H, W))
    y = rng.uniform(0, 1, size=(1, H, W))
    return flat, x, y


def test_network_parameter_count():
    _, n = so.param_layout()
    assert 1_700_000 < n < 2_100_000     # about 2M parameters


def test_network_gradient_matches_finite_differences():
    """Without bf16 rounding the network is piecewise linear; central
    differences on random parameters of every layer pin the backward pass
    (skip copies, upsampling adjoint, strides, head)."""
    flat, x, y = _small_problem()
    loss, g, _ = so.loss_and_grads(flat, x, y, rounding=False)
    layout, _ = so.param_layout()
    rng = np.random.default_rng(7)
    eps = 1e-6
    checked = 0
    for name, o, shape in layout:
        size = int(np.prod(shape))
        for idx in rng.choice(size, size=min(3, size), replace=False):
            i = o + int(idx)
            fp, fm = flat.copy(), flat.copy()
            fp[i] += eps
            fm[i] -= eps
            lp = so.loss_and_grads(fp, x, y, rounding=False)[0]
            lm = so.loss_and_grads(fm, x, y, rounding=False)[0]
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (name, idx, fd, g[i])
            checked += 1
    assert checked > 50


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    w = rng.standard_normal(100)
    g = rng.standard_normal(100)
    w1, m, v = so.adam_update(w, g, np.zeros(100), np.zeros(100), step=1, lr=1e-3)
    # with zero moments the first bias-corrected step is lr * g / (|g| + eps)
    assert np.allclose(w1, w - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_forward_shapes_and_psnr():
    flat, x, y = _small_problem(H=32, W=16)
    act, yhat = so.forward(so.unflatten(flat), x)
    assert yhat.shape == (1, 32, 16)
    assert act["B4"].shape == (1, 2, 1, 256) and act["S0"].shape == (1, 32, 16, 24)
    assert so.psnr(y, y) == 200.0
    assert abs(so.psnr(np.full_like(y, 0.5), np.full_like(y, 0.6)) - 20.0) < 1e-9


def test_depth_integral_definition_and_adjoint():
    """The depth integral is the running sum over the rows strictly above a
    pixel (brute force), and the backward helper is its exact adjoint."""
    rng = np.random.default_rng(5)
    p = rng.standard_normal((2, 7, 3, 4))
    a = so.depth_sum_above(p)
    for y in range(7):
        assert np.allclose(a[:, y], p[:, :y].sum(axis=1), rtol=0, atol=1e-12)
    g = rng.standard_normal(p.shape)
    b = so.depth_sum_below(g)
    for v in range(7):
        assert np.allclose(b[:, v], g[:, v + 1:].sum(axis=1), rtol=0, atol=1e-12)
    assert abs(np.sum(a * g) - np.sum(p * b)) < 1e-10


def test_depth_integral_reaches_the_output_from_above_only():
    """A change of E0 features at one row can move the decoder's appended
    integral channels only in rows below it (causality along the beam)."""
    flat, x, _ = _small_problem(H=32, W=16)
    params = so.unflatten(flat)
    act, _ = so.forward(params, x, rounding=False)
    p = act["E0"] @ params["wp"].T + params["bp"]
    a = so.SCAN_SCALE * so.depth_sum_above(p)
    assert np.allclose(act["S0"][..., -so.SCAN_C:], a)
    p2 = p.copy()
    p2[:, 20] += 1.0
    a2 = so.SCAN_SCALE * so.depth_sum_above(p2)
    assert np.array_equal(a2[:, :21], a[:, :21])
    assert np.allclose(a2[:, 21:] - a[:, 21:], so.SCAN_SCALE)


def test_histogram_matching_lut_pins():
    """Histogram specification: identical histograms map every occupied bin to
    itself; a shifted histogram maps back by the shift; the matched frame's
    cumulative counts never fall below the reference's at the mapped bins."""
    rng = np.random.default_rng(8)
    h = np.bincount(rng.integers(100, 900, 5000), minlength=so.CT_BINS)
    lut = so.histogram_match_lut(h, h)
    occ = np.nonzero(h)[0]
    assert np.array_equal(lut[occ], occ)
    shifted = np.roll(h, 37)
    lut2 = so.histogram_match_lut(shifted, h)
    assert np.array_equal(lut2[occ + 37], occ)
    # monotone, and exact in integers for arbitrary totals
    src = np.bincount(rng.integers(0, 4096, 777), minlength=so.CT_BINS)
    lut3 = so.histogram_match_lut(src, h)
    assert np.all(np.diff(lut3) >= 0)
    sc, rc = np.cumsum(src), np.cumsum(h)
    for b in range(0, 4096, 97):
        r = lut3[b]
        assert rc[r] * sc[-1] >= sc[b] * rc[-1]
        assert r == 0 or rc[r - 1] * sc[-1] < sc[b] * rc[-1]


def test_ct_input_channels():
    """CT input of an axis-aligned frame over a CT volume: channel 0 equals the
    matched nearest HU / 1000 (here matched to the frame's own histogram, so
    unchanged), channels 1-2 the voxel's noise draws, channel 3 the depth."""
    import synth
    from cases import axis_pose
    rng = np.random.default_rng(3)
    lab = np.ones((30, 20, 25), dtype=np.uint8)
    lab[15:] = 3
    ct = synth.ct_from_labels(lab, 5)
    vol = synth.Volume(labels=lab, ct=ct, seed=11)
    probe = synth.Probe(W=12, H=40, dx=1.0, dy=1.0)
    pose = axis_pose((12.0, 9.0, 0.0))
    bins = so.ct_bins(vol, probe, pose)
    x = so.ct_input(vol, probe, pose, so.ct_histogram(bins))
    # pixel (x, y) lies at volume mm (6.5 + x, 9, y): nearest voxel (7 + x, 9, y), rounding half up
    hu = np.full((40, 12), -1000, dtype=np.int64)
    hu[:30] = ct[:30, 9, 7:19]
    expect0 = so.bf16_round((np.clip(hu + 1024, 0, 4095) - 1024).astype(np.float32) / np.float32(1000.0))
    assert np.array_equal(x[..., 0], expect0)
    assert np.all(x[30:, :, 1:3] == 0) and np.all(x[..., 4:] == 0)
    assert abs(x[:30, :, 1].std() - 1.0) < 0.3 and abs(x[:30, :, 2].std() - 1.0) < 0.3
    assert np.array_equal(x[:, 0, 3], so.bf16_round((np.arange(40) + 0.5) / 40))
