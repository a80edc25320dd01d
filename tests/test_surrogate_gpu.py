"""Surrogate kernels and model through the C ABI vs the FP64 oracle (GPU)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import surrogate as so

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
U = 2.0 ** -24   # FP32 unit roundoff: products of bf16 are exact in FP32


@pytest.fixture(scope="module")
def sess():
    from paper_2507_01152_amd.session import Session
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = Session(0)
    yield s
    s.close()


def dev_bf16(a):
    return torch.from_numpy(so.f64_to_bf16_bits(a).view(np.int16)).cuda()


def host_bf16(t):
    return so.bf16_bits_to_f64(t.cpu().numpy().view(np.uint16))


CONV_CASES = [
    # N, H, W, C, Co, k, stride, pad, up
    (2, 16, 12, 8, 16, 3, 1, 1, 0),
    (1, 13, 17, 16, 32, 3, 2, 1, 0),     # ragged output tiles
    (2, 8, 6, 32, 64, 3, 1, 1, 1),       # upsampled input
    (1, 9, 7, 64, 128, 3, 2, 1, 0),
    (1, 5, 4, 256, 256, 3, 1, 1, 0),
    (1, 4, 3, 128, 64, 3, 1, 1, 1),
    (3, 11, 5, 24, 40, 1, 1, 0, 0),      # 1x1, channel counts not powers of two
    (2, 9, 70, 16, 8, 1, 1, 0, 0),       # 1x1 to 8 channels (the depth map), K below one MFMA step
    (2, 7, 9, 64, 32, 1, 1, 0, 0),       # 1x1, two K steps of one tap's 32 channels each
    (2, 7, 9, 48, 24, 1, 1, 0, 0),       # 1x1, two K steps, the second half past K
    (1, 12, 10, 24, 16, 3, 1, 1, 0),     # 24 input channels (the last decoder conv)
    # LDS-tiled direct 3x3 path (stride 1, pad 1, C <= 32, Co 16 or 32): 16 x 32 tiles
    (2, 19, 70, 16, 16, 3, 1, 1, 0),     # ragged tiles in both directions
    (1, 7, 11, 32, 16, 3, 1, 1, 1),      # upsampled to 14 x 22
    (2, 10, 33, 16, 32, 3, 1, 1, 0),     # 32 output channels
    (1, 9, 40, 32, 32, 3, 1, 1, 1),      # upsampled, 32 -> 32
    # upsampled inputs staged as coarse tiles (10 x 18 stored pixels per 16 x 32 output tile)
    (2, 6, 20, 64, 32, 3, 1, 1, 1),      # 64 -> 32 (the U1 shape), ragged tiles in both directions
    (1, 13, 9, 32, 16, 3, 1, 1, 1),      # 32 -> 16 (the U0 shape), odd stored sizes
    # more 8 x 32 weight-gradient tiles than its 512 blocks: blocks accumulate several tiles
    (20, 48, 130, 8, 16, 3, 1, 1, 0),    # 600 tiles, ragged last column tile
    (8, 40, 100, 32, 32, 3, 1, 1, 1),    # upsampled to 80 x 200: 560 tiles
    # wider layers: the direct weight gradient in groups of 32 input x 32 output channels
    (2, 10, 20, 64, 32, 3, 1, 1, 1),     # 2 input groups, upsampled (the U1 shape)
    (1, 12, 33, 64, 64, 3, 1, 1, 0),     # 2 x 2 groups, ragged tiles
    (1, 6, 10, 128, 64, 3, 1, 1, 1),     # 4 x 2 groups, upsampled to 12 x 20 (the U2 shape)
    (2, 9, 16, 96, 96, 3, 1, 1, 0),      # 3 x 3 groups, outputs exactly 16 wide
    (8, 48, 96, 64, 64, 3, 1, 1, 0),     # 144 tiles over 128 blocks per group pair
    # stride 2 with even input sizes: the data gradient as a tiled conv over dy dilated by zeros
    (2, 16, 40, 16, 32, 3, 2, 1, 0),     # the T2 shape
    (1, 22, 70, 16, 32, 3, 2, 1, 0),     # ragged tiles of the 22 x 70 input gradient
    (1, 12, 36, 32, 16, 3, 2, 1, 0),     # 32 input channels, 16 output
    # wider stride-2 layers: the data gradient as one GEMM per output parity class (odd sizes above)
    (2, 16, 24, 32, 64, 3, 2, 1, 0),     # the T3 shape
    # stride-2 weight gradients on the direct kernel (4 x 32 output tiles, even and odd input columns)
    (1, 10, 40, 64, 64, 3, 2, 1, 0),     # 2 x 2 channel groups
    (64, 40, 96, 16, 32, 3, 2, 1, 0),    # 640 tiles over 512 blocks
    # the most channels a conv takes (4096): implicit-GEMM K steps of one tap's 32 channels, every
    # pixel of a 3 x 3 image with padding taps read from the zero source at channel offsets up to C
    (1, 3, 3, 4096, 16, 3, 1, 1, 0),     # forward over 1152 K steps
    (1, 3, 3, 16, 4096, 3, 1, 1, 0),     # data gradient over 4096 output channels
]


@pytest.mark.parametrize("case", CONV_CASES)
def test_conv_forward_parity(sess, case):
    from paper_2507_01152_amd import sonosim as sg
    N, H, W, C, Co, k, st, pad, up = case
    rng = np.random.default_rng(sum(case))
    x = so.bf16_round(rng.standard_normal((N, H, W, C)))
    w = so.bf16_round(rng.standard_normal((Co, k, k, C)) * 0.2)
    b = rng.standard_normal(Co).astype(np.float32).astype(np.float64)
    ref = so.conv_forward(x, w, b, stride=st, pad=pad, up=up, relu=True)
    mag = so.conv_forward(np.abs(x), np.abs(w), np.abs(b), stride=st, pad=pad, up=up)
    skip = so.bf16_round(rng.standard_normal(ref.shape))
    y = torch.empty(ref.shape, dtype=torch.int16, device="cuda")
    ys = torch.empty_like(y)
    yf = torch.empty(ref.shape, dtype=torch.float32, device="cuda")
    d = sg.conv_desc(N, H, W, C, Co, k, st, pad, up)
    sg.sg_conv_forward(sess.ctx, d, dev_bf16(x), dev_bf16(w), torch.tensor(b, dtype=torch.float32, device="cuda"),
                       True, dev_bf16(skip), y, ys, yf)
    torch.cuda.synchronize()
    K = k * k * C
    tol = (K + 2) * U * mag + 1e-30
    got = yf.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= tol)
    # the bf16 output is the FP32 value rounded; the skip output adds in bf16
    assert np.array_equal(host_bf16(y), so.bf16_round(got))
    assert np.array_equal(host_bf16(ys), so.bf16_round(so.bf16_round(got) + skip))


@pytest.mark.parametrize("case", CONV_CASES)
def test_conv_backward_parity(sess, case):
    from paper_2507_01152_amd import sonosim as sg
    N, H, W, C, Co, k, st, pad, up = case
    rng = np.random.default_rng(100 + sum(case))
    x = so.bf16_round(rng.standard_normal((N, H, W, C)))
    w = so.bf16_round(rng.standard_normal((Co, k, k, C)) * 0.2)
    y_shape = so.conv_forward(x, w, stride=st, pad=pad, up=up).shape
    dy = so.bf16_round(rng.standard_normal(y_shape))
    d = sg.conv_desc(N, H, W, C, Co, k, st, pad, up)
    # data gradient, written then accumulated
    dx_ref = so.conv_backward_data(dy, w, x.shape, stride=st, pad=pad, up=up)
    dx_mag = so.conv_backward_data(np.abs(dy), np.abs(w), x.shape, stride=st, pad=pad, up=up)
    dx = torch.empty(x.shape, dtype=torch.float32, device="cuda")
    sg.sg_conv_backward_data(sess.ctx, d, dev_bf16(dy), dev_bf16(w), dx, False)
    torch.cuda.synchronize()
    Kd = k * k * Co * (4 if up else 1)
    got = dx.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - dx_ref) <= (Kd + 2) * U * dx_mag + 1e-30)
    sg.sg_conv_backward_data(sess.ctx, d, dev_bf16(dy), dev_bf16(w), dx, True)
    torch.cuda.synchronize()
    got2 = dx.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got2 - 2 * dx_ref) <= 2 * (Kd + 3) * U * dx_mag + 1e-30)
    # weight and bias gradients
    dw_ref, db_ref = so.conv_backward_weight(x, dy, k=k, stride=st, pad=pad, up=up)
    dw_mag, db_mag = so.conv_backward_weight(np.abs(x), np.abs(dy), k=k, stride=st, pad=pad, up=up)
    dw = torch.empty(w.shape, dtype=torch.float32, device="cuda")
    # (the bias gradient takes at most 256 channels; the entry point rejects more)
    db = torch.empty(Co, dtype=torch.float32, device="cuda") if Co <= 256 else None
    sg.sg_conv_backward_weight(sess.ctx, d, dev_bf16(x), dev_bf16(dy), dw, db)
    torch.cuda.synchronize()
    Kw = int(np.prod(y_shape[:3]))
    assert np.all(np.abs(dw.cpu().numpy() - dw_ref) <= (Kw + 2) * U * dw_mag + 1e-30)
    if db is not None:
        assert np.all(np.abs(db.cpu().numpy() - db_ref) <= (Kw + 2) * U * db_mag + 1e-30)
    # deterministic: a second run is bit-identical
    dw2 = torch.empty_like(dw)
    sg.sg_conv_backward_weight(sess.ctx, d, dev_bf16(x), dev_bf16(dy), dw2, None)
    torch.cuda.synchronize()
    assert torch.equal(dw, dw2)


def _pairs(n, H, W, seed):
    """n envs on 64^3 ellipsoid phantoms imaged at H x W (0.25 mm pixels)."""
    return synth.ellipsoid_workload(seed=seed, n_envs=n, W=W, H=H, dx=0.25, dy=0.25)


def test_encoder_channels_match_oracle(sess):
    from paper_2507_01152_amd import sonosim as sg
    H, W = 48, 32
    wl = _pairs(2, H, W, seed=21)
    vids = sess.load(wl)
    sid = sg.sg_surr_create(sess.ctx, H, W, seed=1)
    sg.sg_surr_train_step(sess.ctx, sid, vids, wl.probes, wl.poses, 0.0)
    xin, _ = sg.sg_surr_get_batch(sess.ctx, sid, 2, H, W)
    x = so.bf16_bits_to_f64(xin)
    t1 = wl.table.copy()
    t1[:, 2] = 0.0   # mu0 = 0, sigma0 = 1: the oracle's T is the gated N0
    t1[:, 3] = 1.0
    for e in range(2):
        o = oracle.simulate_env(wl.volumes[e], t1, wl.probes[e], wl.poses[e], planes=("label", "T"))
        onehot = np.eye(4)[o["label"]]
        assert np.array_equal(x[e, :, :, :4], onehot)
        depth = so.bf16_round((np.arange(H) + 0.5) / H)
        assert np.array_equal(x[e, :, :, 5], np.broadcast_to(depth[:, None], (H, W)))
        assert np.all(x[e, :, :, 6:] == 0)
        ref = o["T"]
        assert np.array_equal(x[e, :, :, 4] != 0, ref != 0)
        # within one bf16 step of the FP64 value
        assert np.all(np.abs(x[e, :, :, 4] - ref) <= 2.0 ** -7 * np.abs(ref) + 1e-6)
    sg.sg_surr_destroy(sess.ctx, sid)


def _label_problem(seed, n, H, W):
    """Seeded parameters and label-mode input pairs (one-hot label, gated
    scatterer sample, depth) with a target that depends on them."""
    rng = np.random.default_rng(seed)
    layout, ng = so.param_layout()
    g = np.zeros(ng)
    for name, o, shape in layout:
        sz = int(np.prod(shape))
        if name.startswith("w") or name in ("wp", "head_w"):
            fan = int(np.prod(shape[1:])) if len(shape) > 1 else int(shape[0])
            g[o:o + sz] = rng.standard_normal(sz) * np.sqrt(2.0 / fan)
        else:
            g[o:o + sz] = rng.standard_normal(sz) * 0.02
    x = np.zeros((n, H, W, 8))
    lab = rng.integers(0, 4, size=(n, H, W))
    x[..., :4] = np.eye(4)[lab]
    x[..., 4] = so.bf16_round(np.where(rng.uniform(size=(n, H, W)) < 0.3, rng.standard_normal((n, H, W)), 0.0))
    x[..., 5] = so.bf16_round((np.arange(H) + 0.5) / H)[None, :, None]
    y = np.clip(0.2 * lab + 0.1 * x[..., 4] + 0.05 * rng.standard_normal((n, H, W)), 0, 1).astype(np.float32)
    return g.astype(np.float32), x, y


def test_training_gradients_match_oracle(sess):
    """Every layer's gradient of one training step against the FP64 network
    oracle on the same seeded parameters, bf16 input and target (given to the
    library through sg_surr_train_pairs).  bf16 rounding flips of single
    activations (FP32 vs FP64 sums) make the layers differ by about 1e-3 to
    1e-2 in norm.  The flips matter most in the deepest levels, which have
    the fewest pixels, so the batch is 4 frames of 128 x 64 (8 x 4 at the
    bottleneck); the noise falls as one over the root of the pixel count."""
    from paper_2507_01152_amd import sonosim as sg
    H, W, n = 128, 64, 4
    p0, x, y = _label_problem(5, n, H, W)
    xin = torch.from_numpy(so.f64_to_bf16_bits(x).view(np.int16)).cuda()
    tgt = torch.from_numpy(y).cuda()
    sid = sg.sg_surr_create(sess.ctx, H, W, seed=11)
    sg.sg_surr_set_params(sess.ctx, sid, p0)
    loss = sg.sg_surr_train_pairs(sess.ctx, sid, xin, tgt, 0.0)
    g = sg.sg_surr_get_grads(sess.ctx, sid).astype(np.float64)
    ref_loss, ref_g, _ = so.loss_and_grads(p0.astype(np.float64), x, y.astype(np.float64))
    assert abs(loss - ref_loss) <= 1e-3 * ref_loss
    layout, _ = so.param_layout()
    report = []
    for name, o, shape in layout:
        sz = int(np.prod(shape))
        a, b = g[o:o + sz], ref_g[o:o + sz]
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        cos = float(a @ b) / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30)
        report.append((name, round(float(err), 5), round(cos, 6)))
    print(report)
    bad = [r for r in report if not (r[1] <= 2e-2 and r[2] >= 0.999)]
    assert not bad, bad
    # one Adam step from zero moments moves each weight by lr * g / (|g| + eps)
    lr = 1e-3
    sid2 = sg.sg_surr_create(sess.ctx, H, W, seed=11)
    sg.sg_surr_set_params(sess.ctx, sid2, p0)
    sg.sg_surr_train_pairs(sess.ctx, sid2, xin, tgt, lr)
    g2 = sg.sg_surr_get_grads(sess.ctx, sid2).astype(np.float64)
    p1 = sg.sg_surr_get_params(sess.ctx, sid2).astype(np.float64)
    assert np.array_equal(g2, g)   # the same batch gives the same gradient
    expect = p0 - lr * g2 / (np.abs(g2) + 1e-8)
    # FP32 bias corrections (0.999 is not exact in FP32) allow ~1e-5 relative
    assert np.allclose(p1, expect, rtol=1e-4, atol=1e-6 * lr)
    sg.sg_surr_destroy(sess.ctx, sid)
    sg.sg_surr_destroy(sess.ctx, sid2)


def test_encoded_pairs_train_like_given_pairs(sess):
    """sg_surr_train_step (encoder + physics) and sg_surr_train_pairs on the
    batch it encoded and rendered give the same step, bit for bit."""
    from paper_2507_01152_amd import sonosim as sg
    H, W, n = 64, 32, 2
    wl = _pairs(n, H, W, seed=5)
    vids = sess.load(wl)
    a = sg.sg_surr_create(sess.ctx, H, W, seed=3)
    b = sg.sg_surr_create(sess.ctx, H, W, seed=3)
    la = sg.sg_surr_train_step(sess.ctx, a, vids, wl.probes, wl.poses, 1e-3)
    xin, tgt = sg.sg_surr_get_batch(sess.ctx, a, n, H, W)
    lb = sg.sg_surr_train_pairs(sess.ctx, b, torch.from_numpy(xin.view(np.int16)).cuda(),
                                torch.from_numpy(tgt).cuda(), 1e-3)
    assert la == lb
    assert np.array_equal(sg.sg_surr_get_params(sess.ctx, a), sg.sg_surr_get_params(sess.ctx, b))
    for s in (a, b):
        sg.sg_surr_destroy(sess.ctx, s)


def _random_pairs(n, H, W, seed):
    rng = np.random.default_rng(seed)
    xin = torch.from_numpy(so.bf16_round(rng.random((n, H, W, 8))).astype(np.float32)).to(torch.bfloat16)
    tgt = torch.from_numpy(rng.random((n, H, W)).astype(np.float32))
    return xin.view(torch.int16).cuda(), tgt.cuda()


@pytest.mark.parametrize("adv", [0.0, 0.01])
def test_graph_replay_matches_eager_bit_for_bit(sess, adv):
    """The captured training step (first step of a batch size eager, the
    second captured, later ones replayed) gives the same losses, parameters
    and discriminator state as kernel-by-kernel steps, also when the batch
    size changes and the graph is captured again."""
    from paper_2507_01152_amd import sonosim as sg
    H, W = 32, 48
    mk = (lambda: sg.sg_surr_create_ct(sess.ctx, H, W, seed=4, adv_weight=adv)) if adv else \
        (lambda: sg.sg_surr_create(sess.ctx, H, W, seed=4))
    eager, graph = mk(), mk()
    sg.sg_surr_set_graph(sess.ctx, eager, False)
    batches = [_random_pairs(n, H, W, 60 + i) for i, n in enumerate([3, 3, 3, 3, 2, 2, 2, 3, 3])]
    for xin, tgt in batches:
        la = sg.sg_surr_train_pairs(sess.ctx, eager, xin, tgt, 2e-3)
        lb = sg.sg_surr_train_pairs(sess.ctx, graph, xin, tgt, 2e-3)
        assert la == lb
        if adv:
            assert sg.sg_surr_gan_losses(sess.ctx, eager) == sg.sg_surr_gan_losses(sess.ctx, graph)
    assert np.array_equal(sg.sg_surr_get_params(sess.ctx, eager), sg.sg_surr_get_params(sess.ctx, graph))
    if adv:
        assert np.array_equal(sg.sg_surr_disc_get_params(sess.ctx, eager), sg.sg_surr_disc_get_params(sess.ctx, graph))
    for s in (eager, graph):
        sg.sg_surr_destroy(sess.ctx, s)


def test_async_steps_keep_their_losses_on_the_device(sess):
    """Enqueued steps (no readback) give the steps and losses of synchronous
    ones; the device keeps the last 4096 steps' losses, read across the
    ring's wrap."""
    from paper_2507_01152_amd import sonosim as sg
    H, W = 32, 48
    a = sg.sg_surr_create(sess.ctx, H, W, seed=8)
    b = sg.sg_surr_create(sess.ctx, H, W, seed=8)
    batches = [_random_pairs(2, H, W, 70 + i) for i in range(6)]
    want = [sg.sg_surr_train_pairs(sess.ctx, a, xin, tgt, 1e-3) for xin, tgt in batches]
    for xin, tgt in batches:
        sg.sg_surr_train_pairs_async(sess.ctx, b, xin, tgt, 1e-3)
    assert sg.sg_surr_step_count(sess.ctx, b) == 6
    hist = sg.sg_surr_loss_history(sess.ctx, b, 1, 6)
    assert list(hist[:, 0]) == want and not hist[:, 1:].any()
    assert np.array_equal(sg.sg_surr_get_params(sess.ctx, a), sg.sg_surr_get_params(sess.ctx, b))
    with pytest.raises(sg.SonosimError):
        sg.sg_surr_loss_history(sess.ctx, b, 6, 2)   # step 7 not enqueued
    # across the ring's end: 4098 steps of a tiny network
    c = sg.sg_surr_create(sess.ctx, 16, 16, seed=9)
    xin, tgt = _random_pairs(1, 16, 16, 80)
    for _ in range(4097):
        sg.sg_surr_train_pairs_async(sess.ctx, c, xin, tgt, 1e-4)
    last = sg.sg_surr_train_pairs(sess.ctx, c, xin, tgt, 1e-4)
    h = sg.sg_surr_loss_history(sess.ctx, c, 4094, 5)
    assert h[-1, 0] == last and np.all(np.isfinite(h))
    assert np.array_equal(h[:, 0], sg.sg_surr_loss_history(sess.ctx, c, 4094, 5)[:, 0])
    with pytest.raises(sg.SonosimError):
        sg.sg_surr_loss_history(sess.ctx, c, 2, 1)   # older than the last 4096 steps
    for s in (a, b, c):
        sg.sg_surr_destroy(sess.ctx, s)


def test_checkpoint_resume_is_bit_exact(sess, tmp_path):
    from paper_2507_01152_amd import sonosim as sg
    H, W = 32, 48
    wl = _pairs(3, H, W, seed=8)
    vids = sess.load(wl)
    sid = sg.sg_surr_create(sess.ctx, H, W, seed=3)
    for _ in range(2):
        sg.sg_surr_train_step(sess.ctx, sid, vids, wl.probes, wl.poses, 1e-3)
    path = str(tmp_path / "ck.bin")
    sg.sg_surr_save(sess.ctx, sid, path)
    la = [sg.sg_surr_train_step(sess.ctx, sid, vids, wl.probes, wl.poses, 1e-3) for _ in range(2)]
    pa = sg.sg_surr_get_params(sess.ctx, sid)
    sid2 = sg.sg_surr_create(sess.ctx, H, W, seed=99)
    sg.sg_surr_load(sess.ctx, sid2, path)
    lb = [sg.sg_surr_train_step(sess.ctx, sid2, vids, wl.probes, wl.poses, 1e-3) for _ in range(2)]
    pb = sg.sg_surr_get_params(sess.ctx, sid2)
    assert la == lb and np.array_equal(pa, pb)
    bad = sg.sg_surr_create(sess.ctx, 48, 48, seed=1)
    with pytest.raises(sg.SonosimError):
        sg.sg_surr_load(sess.ctx, bad, path)


def test_training_reduces_loss(sess):
    from paper_2507_01152_amd import sonosim as sg
    H, W = 64, 32
    wl = _pairs(8, H, W, seed=13)
    vids = sess.load(wl)
    sid = sg.sg_surr_create(sess.ctx, H, W, seed=5)
    losses = [sg.sg_surr_train_step(sess.ctx, sid, vids, wl.probes, wl.poses, 2e-3) for _ in range(60)]
    assert np.mean(losses[-5:]) < 0.7 * np.mean(losses[:3])


def test_infer_audit_and_fallback(sess):
    from paper_2507_01152_amd import sonosim as sg
    H, W, n = 64, 32, 12
    wl = _pairs(n, H, W, seed=17)
    vids = sess.load(wl)
    sid = sg.sg_surr_create(sess.ctx, H, W, seed=2)
    for _ in range(20):
        sg.sg_surr_train_step(sess.ctx, sid, vids, wl.probes, wl.poses, 2e-3)
    phys, offs, _ = sess.simulate(wl, vids)
    phys = phys.cpu().numpy().reshape(n, H, W)
    out = torch.empty(n * H * W, dtype=torch.float32, device="cuda")
    audit = [1, 4, 7, 10]
    # no audit: pure network output, clamped
    _, nf = sg.sg_surr_infer(sess.ctx, sid, vids, wl.probes, wl.poses, out, [], 30.0)
    net = out.cpu().numpy().reshape(n, H, W)
    assert nf == 0 and net.min() >= 0 and net.max() <= 1
    # audit that never fails: frames unchanged, PSNR as computed on the host
    psnr, nf = sg.sg_surr_infer(sess.ctx, sid, vids, wl.probes, wl.poses, out, audit, -np.inf, 0.25)
    assert nf == 0 and np.array_equal(out.cpu().numpy().reshape(n, H, W), net)
    for i, e in enumerate(audit):
        assert abs(psnr[i] - so.psnr(net[e], phys[e])) < 1e-3
    # a threshold between the audited PSNRs: failing frames come from physics
    thr = float(np.median(psnr))
    psnr2, nf = sg.sg_surr_infer(sess.ctx, sid, vids, wl.probes, wl.poses, out, audit, thr, 1.0)
    got = out.cpu().numpy().reshape(n, H, W)
    fails = [e for p, e in zip(psnr2, audit) if not p >= thr]
    assert nf == len(fails) and 0 < nf < len(audit)
    for e in range(n):
        assert np.array_equal(got[e], phys[e] if e in fails else net[e])
    # every audited frame failing beyond the allowed fraction: whole step from physics
    _, nf = sg.sg_surr_infer(sess.ctx, sid, vids, wl.probes, wl.poses, out, audit, np.inf, 0.25)
    assert nf == n and np.array_equal(out.cpu().numpy().reshape(n, H, W), phys)
    with pytest.raises(sg.SonosimError):
        sg.sg_surr_infer(sess.ctx, sid, vids, wl.probes, wl.poses, out, [1, 1], 30.0)


def test_trained_network_gains_over_untrained_and_lookup(sess):
    """What the learned network adds: on held-out phantoms its frames must
    beat (a) the same network untrained and (b) the best non-learned
    predictor built from the same inputs, a lookup of the mean physics value
    per (label, depth row) measured on the training pairs."""
    from paper_2507_01152_amd import sonosim as sg
    from paper_2507_01152_amd.train_surrogate import PairSource
    H, W, B = 256, 128, 32
    train_src = PairSource(sess, 64, seed0=0)
    test_src = PairSource(sess, 16, seed0=300000)
    sid = sg.sg_surr_create(sess.ctx, H, W, seed=4)
    rng = np.random.default_rng(0)
    vids, probes, poses = test_src.batch(32, np.random.default_rng(99))
    out = torch.empty(32 * H * W, dtype=torch.float32, device="cuda")
    audit = list(range(32))
    psnr_init, _ = sg.sg_surr_infer(sess.ctx, sid, vids, probes, poses, out, audit, -np.inf, 1.0)
    # lookup table from training pairs: mean target per (label, row)
    acc = np.zeros((4, H))
    cnt = np.zeros((4, H))
    for step in range(600):
        v, p, q = train_src.batch(B, rng)
        sg.sg_surr_train_step(sess.ctx, sid, v, p, q, 5e-4)
        if step % 50 == 0:
            xin, tgt = sg.sg_surr_get_batch(sess.ctx, sid, B, H, W)
            lab = so.bf16_bits_to_f64(xin[..., :4]).argmax(-1)
            for l in range(4):
                m = lab == l
                acc[l] += (tgt * m).sum(axis=(0, 2))
                cnt[l] += m.sum(axis=(0, 2))
    table = acc / np.maximum(cnt, 1)
    psnr_net, _ = sg.sg_surr_infer(sess.ctx, sid, vids, probes, poses, out, audit, -np.inf, 1.0)
    # the lookup baseline on the same held-out frames (labels from the encoder);
    # a zero-rate step only encodes and renders them
    sg.sg_surr_train_step(sess.ctx, sid, vids, probes, poses, 0.0)   # encode + render the held-out envs
    xin, tgt = sg.sg_surr_get_batch(sess.ctx, sid, 32, H, W)
    lab = so.bf16_bits_to_f64(xin[..., :4]).argmax(-1)
    look = table[lab, np.arange(H)[None, :, None]]
    psnr_look = [so.psnr(look[i], tgt[i]) for i in range(32)]
    gain_init = float(np.mean(psnr_net) - np.mean(psnr_init))
    gain_look = float(np.mean(psnr_net) - np.mean(psnr_look))
    print(f"held-out PSNR: trained {np.mean(psnr_net):.2f} dB, untrained {np.mean(psnr_init):.2f} dB, "
          f"lookup {np.mean(psnr_look):.2f} dB")
    assert gain_init > 5.0 and gain_look > 2.0
    sg.sg_surr_destroy(sess.ctx, sid)


def test_inference_at_full_size_vs_oracle(sess):
    """Inference of 1024 envs of 128 x 256 frames (the benchmark's surrogate
    workload size, in the same call) on seeded parameters: two sampled envs'
    outputs against the FP64 network oracle on the oracle's own encoding of
    those envs (one-hot label, gated N0 rounded to bf16, depth; the library's
    N0 is within one bf16 step of it).  The head is scaled to 0.1 with bias
    0.5 so that the clamped output keeps the network's variation; the network
    part (output - 0.5) is compared where neither side clamps, with the bar of
    the gradient test (bf16 rounding flips of FP32 vs FP64 sums)."""
    from paper_2507_01152_amd import sonosim as sg
    H, W, n = 256, 128, 1024
    p0, _, _ = _label_problem(7, 1, 16, 16)
    layout, _ = so.param_layout()
    off = {name: (o, shape) for name, o, shape in layout}
    o, shape = off["head_w"]
    p0[o:o + int(np.prod(shape))] *= 0.1
    p0[off["head_b"][0]] = 0.5
    wl = _pairs(n, H, W, seed=31)
    vids = sess.load(wl)
    sid = sg.sg_surr_create(sess.ctx, H, W, seed=3)
    sg.sg_surr_set_params(sess.ctx, sid, p0)
    out = torch.empty(n * H * W, dtype=torch.float32, device="cuda")
    _, nf = sg.sg_surr_infer(sess.ctx, sid, vids, wl.probes, wl.poses, out, [], 30.0)
    assert nf == 0
    net = out.cpu().numpy().reshape(n, H, W).astype(np.float64)
    sg.sg_surr_destroy(sess.ctx, sid)
    pick = [5, 777]
    t1 = wl.table.copy()
    t1[:, 2] = 0.0   # mu0 = 0, sigma0 = 1: the oracle's T is the gated N0
    t1[:, 3] = 1.0
    x = np.zeros((len(pick), H, W, 8))
    for i, e in enumerate(pick):
        o = oracle.simulate_env(wl.volumes[e], t1, wl.probes[e], wl.poses[e], planes=("label", "T"))
        x[i, :, :, :4] = np.eye(4)[o["label"]]
        x[i, :, :, 4] = so.bf16_round(o["T"])
        x[i, :, :, 5] = so.bf16_round((np.arange(H) + 0.5) / H)[:, None]
    _, yhat = so.forward(so.unflatten(p0.astype(np.float64)), x)
    for i, e in enumerate(pick):
        a, b = net[e], yhat[i]
        inside = (a > 0) & (a < 1) & (b > 0) & (b < 1)
        assert inside.mean() > 0.5
        da, db = a[inside] - 0.5, b[inside] - 0.5
        err = np.linalg.norm(da - db) / np.linalg.norm(db)
        cos = float(da @ db) / (np.linalg.norm(da) * np.linalg.norm(db))
        print(e, round(float(err), 5), round(cos, 6))
        assert err <= 2e-2 and cos >= 0.999, (e, err, cos)
