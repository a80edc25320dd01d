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


# ---------------------------------------------------------------------------
# adversarial term (conditional patch discriminator, binary cross-entropy)


def _disc_params(seed=4, scale=1.0):
    rng = np.random.default_rng(seed)
    layout, n = so.disc_layout()
    flat = np.zeros(n)
    for name, o, shape in layout:
        sz = int(np.prod(shape))
        if name.startswith("dw"):
            flat[o:o + sz] = rng.standard_normal(sz) * scale * np.sqrt(2.0 / np.prod(shape[1:]))
        else:
            flat[o:o + sz] = rng.standard_normal(sz) * 0.05
    return flat


def test_softplus_sigmoid_and_bce_closed_forms():
    l = np.array([-1000.0, -30.0, -1.5, 0.0, 0.25, 7.0, 1000.0])
    assert so.softplus(np.array([0.0]))[0] == np.log(2.0)
    # softplus(-l) - softplus(l) = -l, and no overflow at |l| = 1000
    assert np.allclose(so.softplus(-l) - so.softplus(l), -l, rtol=0, atol=1e-12)
    assert so.softplus(np.array([1000.0]))[0] == 1000.0 and so.softplus(np.array([-1000.0]))[0] == 0.0
    assert so.sigmoid(np.array([0.0]))[0] == 0.5
    assert np.allclose(so.sigmoid(l) + so.sigmoid(-l), 1.0, atol=1e-15)
    # d softplus / dl = sigmoid, by central differences
    h = 1e-6
    m = np.abs(l) < 100
    fd = (so.softplus(l[m] + h) - so.softplus(l[m] - h)) / (2 * h)
    assert np.allclose(fd, so.sigmoid(l[m]), atol=1e-8)
    for label in (0, 1):
        v, g = so.bce_logits(l, label)
        assert np.allclose(g, so.sigmoid(l) - label, atol=0)
        assert np.all(v >= 0)
    # label 1 at logit 0 costs log 2; a confident right answer costs ~0
    assert so.bce_logits(np.array([0.0]), 1)[0][0] == np.log(2.0)
    assert so.bce_logits(np.array([50.0]), 1)[0][0] < 1e-20


def test_leaky_relu_values():
    a = np.array([-2.0, -0.0, 0.0, 3.0])
    assert np.array_equal(so.leaky_relu(a), [-2.0 * float(np.float32(0.2)), 0.0, 0.0, 3.0])
    assert so.LEAKY_SLOPE == float(np.float32(0.2))


@pytest.mark.parametrize("chan", [0, so.DISC_IMAGE_C])
def test_disc_forward_center_tap_pin(chan):
    """Each layer passes the centre tap of one channel to channel 0 (weight 1,
    no bias): the logit at patch (i, j) is input pixel (8i, 8j) of that
    channel after four leaky ReLUs, i.e. v for v > 0 and slope^4 v else.
    With chan = 4 the value comes from the image placed by disc_input."""
    layout, n = so.disc_layout()
    dp = so.disc_unflatten(np.zeros(n))
    dp["dw0"][0, 1, 1, chan] = 1.0
    for i in range(1, len(so.DISC_LAYERS)):
        dp[f"dw{i}"][0, 1, 1, 0] = 1.0
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 32, 48, 8))
    img = rng.standard_normal((2, 32, 48))
    z = so.disc_input(x, img, rounding=False)
    assert np.array_equal(z[..., :4], x[..., :4]) and np.array_equal(z[..., 4], img) and not z[..., 5:].any()
    _, logits = so.disc_forward(dp, z, rounding=False)
    v = z[:, ::8, ::8, chan]
    assert logits.shape == (2, 4, 6)
    assert np.allclose(logits, np.where(v > 0, v, so.LEAKY_SLOPE ** 4 * v), rtol=1e-15, atol=0)


def test_disc_backward_matches_finite_differences():
    """Without rounding the discriminator is piecewise linear: central
    differences of sum(c * logits) w.r.t. parameters of every layer and
    input pixels pin the backward (strides, leaky mask, channel-0 logit)."""
    flat = _disc_params(seed=5)
    rng = np.random.default_rng(6)
    z = rng.standard_normal((1, 16, 24, 8))
    c = rng.standard_normal((1, 2, 3))

    def f(fl, zz):
        return float((c * so.disc_forward(so.disc_unflatten(fl), zz, rounding=False)[1]).sum())

    dp = so.disc_unflatten(flat)
    act, _ = so.disc_forward(dp, z, rounding=False)
    grads, dz = so.disc_backward(dp, act, c, rounding=False)
    g = so.disc_flatten(grads)
    eps = 1e-6
    layout, _ = so.disc_layout()
    checked = 0
    for name, o, shape in layout:
        size = int(np.prod(shape))
        for idx in rng.choice(size, size=min(4, size), replace=False):
            i = o + int(idx)
            fp, fm = flat.copy(), flat.copy()
            fp[i] += eps
            fm[i] -= eps
            fd = (f(fp, z) - f(fm, z)) / (2 * eps)
            assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (name, idx, fd, g[i])
            checked += 1
    # the last conv's channels 1..7 carry no gradient
    o = dict((nm, off) for nm, off, _ in layout)["dw4"]
    assert not g[o + 9 * 128:o + 8 * 9 * 128].any()
    for _ in range(8):
        p = tuple(int(rng.integers(0, s)) for s in z.shape)
        zp, zm = z.copy(), z.copy()
        zp[p] += eps
        zm[p] -= eps
        fd = (f(flat, zp) - f(flat, zm)) / (2 * eps)
        assert abs(fd - dz[p]) <= 1e-6 * max(1.0, abs(dz[p])) + 1e-9, (p, fd, dz[p])
        checked += 1
    assert checked >= 28


def test_gan_step_gradients_match_finite_differences():
    """The step's three gradients against central differences of the losses
    they belong to (no rounding, learning rate 0 so the discriminator that
    judges the generator is the one that was differentiated):
    d_grads of L_D at fixed yhat, g_grads of L1 + w L_adv through G and D."""
    gflat, x, y = _small_problem(seed=9)
    x[..., 5:] = 0.0
    dflat = _disc_params(seed=10)
    w = 0.7
    r = so.gan_train_step(gflat, dflat, x, y, w, 0.0, rounding=False)
    assert np.array_equal(r["d_new"], dflat)
    yhat = r["yhat"]

    def loss_d(df):
        dp = so.disc_unflatten(df)
        lr_ = so.disc_forward(dp, so.disc_input(x, y, False), False)[1]
        lf_ = so.disc_forward(dp, so.disc_input(x, yhat, False), False)[1]
        return 0.5 * (so.bce_logits(lr_, 1)[0].mean() + so.bce_logits(lf_, 0)[0].mean())

    def loss_g(gf):
        _, yh = so.forward(so.unflatten(gf), x, rounding=False)
        lg = so.disc_forward(so.disc_unflatten(dflat), so.disc_input(x, yh, False), False)[1]
        return so.l1_loss(yh, y) + w * so.bce_logits(lg, 1)[0].mean()

    assert abs(loss_d(dflat) - r["loss_d"]) <= 1e-12
    rng = np.random.default_rng(11)
    eps = 1e-6
    for i in rng.choice(dflat.size, size=12, replace=False):
        fp, fm = dflat.copy(), dflat.copy()
        fp[i] += eps
        fm[i] -= eps
        fd = (loss_d(fp) - loss_d(fm)) / (2 * eps)
        assert abs(fd - r["d_grads"][i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, r["d_grads"][i])
    layout, _ = so.param_layout()
    adv_seen = 0.0
    for name, o, shape in layout:
        size = int(np.prod(shape))
        for idx in rng.choice(size, size=min(2, size), replace=False):
            i = o + int(idx)
            fp, fm = gflat.copy(), gflat.copy()
            fp[i] += eps
            fm[i] -= eps
            fd = (loss_g(fp) - loss_g(fm)) / (2 * eps)
            assert abs(fd - r["g_grads"][i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (name, idx, fd, r["g_grads"][i])
    # the adversarial term changes the generator's gradient
    g_l1 = so.loss_and_grads(gflat, x, y, rounding=False)[1]
    assert np.linalg.norm(r["g_grads"] - g_l1) > 1e-3 * np.linalg.norm(g_l1)


def test_gan_step_discriminator_update_is_adam():
    gflat, x, y = _small_problem(seed=12)
    x[..., 5:] = 0.0
    dflat = _disc_params(seed=13)
    r = so.gan_train_step(gflat, dflat, x, y, 0.01, 1e-3)
    g = r["d_grads"]
    assert np.allclose(r["d_new"], dflat - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)
    # pix2pix's order: the generator is judged by the updated discriminator
    r2 = so.gan_train_step(gflat, r["d_new"], x, y, 0.01, 0.0)
    assert np.array_equal(r2["g_grads"], r["g_grads"])
    r3 = so.gan_train_step(gflat, dflat, x, y, 0.01, 0.0)
    assert not np.array_equal(r3["g_grads"], r["g_grads"])
