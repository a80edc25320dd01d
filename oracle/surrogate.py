"""FP64 oracle of the learned surrogate (test infrastructure only).

Only the tests, the package's smoke check and the benchmark's CPU-baseline
leg may import this module.  It shares no code with the GPU path.

The surrogate follows the paper's learning-based simulator in spirit
(Sec. 4 and App. B.2: a pix2pix-style encoder-decoder with skip connections
trained with an L1 term): a five-level encoder-decoder on one-hot label
slices plus one scatterer channel.  Numbers are bf16 where the GPU stores
bf16 (weights, activations, the masked output gradients), with every sum
carried out in FP64 here instead of FP32.

The decoder's last 3x3 conv also reads a beam-axis integral: a 1x1 map of
the full-resolution encoder tensor E0 to 8 channels, summed down each
scanline over the rows above the pixel (scaled by 1/16) and appended to S0.
This mirrors the exclusive depth integral of the energy equation (App. B.2),
which a plain encoder-decoder reproduces only coarsely.

Conventions:
  tensors NHWC, rows = depth; conv weights [Co][k][k][Ci]; parameters
  flattened layer by layer as (weights, bias), then the depth-integral map
  (8 x 16 weights, 8 biases), then the 1x1 head (16 weights, 1 bias).
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# bf16 rounding


def bf16_round(x) -> np.ndarray:
    """Nearest bfloat16 value (ties to even) of each element, as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits_to_f64(b) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def f64_to_bf16_bits(x) -> np.ndarray:
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


# ---------------------------------------------------------------------------
# convolution and its two gradients, from the definition
# out[n, ho, wo, co] = sum_{r, s, ci} xpad[n, ho*stride + r, wo*stride + s, ci] * w[co, r, s, ci]


def upsample2(x: np.ndarray) -> np.ndarray:
    """Nearest-neighbour x2 upsampling of NHWC."""
    return x.repeat(2, axis=1).repeat(2, axis=2)


def _out_size(n, k, stride, pad):
    return (n + 2 * pad - k) // stride + 1


def conv_forward(x, w, b=None, stride=1, pad=1, up=False, relu=False):
    x = upsample2(x) if up else x
    N, H, W, C = x.shape
    Co, k = w.shape[0], w.shape[1]
    Ho, Wo = _out_size(H, k, stride, pad), _out_size(W, k, stride, pad)
    xp = np.pad(x, ((0, 0), (pad, pad), (pad, pad), (0, 0)))
    out = np.zeros((N, Ho, Wo, Co))
    for r in range(k):
        for s in range(k):
            patch = xp[:, r:r + stride * (Ho - 1) + 1:stride, s:s + stride * (Wo - 1) + 1:stride, :]
            out += patch @ w[:, r, s, :].T
    if b is not None:
        out += b
    if relu:
        out = np.maximum(out, 0.0)
    return out


def conv_backward_data(dy, w, in_shape, stride=1, pad=1, up=False):
    """Gradient w.r.t. the stored input (N, H, W, C) of conv_forward (no
    activation); with up the four fine positions of each input are summed."""
    N, H, W, C = in_shape
    Hin, Win = (2 * H, 2 * W) if up else (H, W)
    Co, k = w.shape[0], w.shape[1]
    Ho, Wo = dy.shape[1], dy.shape[2]
    dxp = np.zeros((N, Hin + 2 * pad, Win + 2 * pad, C))
    for r in range(k):
        for s in range(k):
            dxp[:, r:r + stride * (Ho - 1) + 1:stride, s:s + stride * (Wo - 1) + 1:stride, :] += dy @ w[:, r, s, :]
    dx = dxp[:, pad:pad + Hin, pad:pad + Win, :]
    if up:
        dx = dx.reshape(N, H, 2, W, 2, C).sum(axis=(2, 4))
    return dx


def conv_backward_weight(x, dy, k=3, stride=1, pad=1, up=False):
    """(dw [Co][k][k][C], db [Co]) of conv_forward for output gradient dy."""
    x = upsample2(x) if up else x
    N, H, W, C = x.shape
    Co = dy.shape[3]
    Ho, Wo = dy.shape[1], dy.shape[2]
    xp = np.pad(x, ((0, 0), (pad, pad), (pad, pad), (0, 0)))
    g = dy.reshape(-1, Co)
    dw = np.zeros((Co, k, k, C))
    for r in range(k):
        for s in range(k):
            patch = xp[:, r:r + stride * (Ho - 1) + 1:stride, s:s + stride * (Wo - 1) + 1:stride, :]
            dw[:, r, s, :] = g.T @ patch.reshape(-1, C)
    return dw, dy.sum(axis=(0, 1, 2))


# ---------------------------------------------------------------------------
# the network

# tensor name -> (channels, pyramid level)
TENSORS = {
    "X": (8, 0), "T1": (16, 0), "E0": (16, 0), "T2": (32, 1), "E1": (32, 1), "T3": (64, 2), "E2": (64, 2),
    "T4": (128, 3), "E3": (128, 3), "T5": (256, 4), "B4": (256, 4),
    "U3": (128, 3), "S3": (128, 3), "D3": (128, 3), "U2": (64, 2), "S2": (64, 2), "D2": (64, 2),
    "U1": (32, 1), "S1": (32, 1), "D1": (32, 1), "U0": (16, 0), "S0": (24, 0), "D0": (16, 0),
}

# (input, output, stride, upsample, skip tensor, skip-added output); all 3x3, pad 1, ReLU
LAYERS = [
    ("X", "T1", 1, False, None, None), ("T1", "E0", 1, False, None, None),
    ("E0", "T2", 2, False, None, None), ("T2", "E1", 1, False, None, None),
    ("E1", "T3", 2, False, None, None), ("T3", "E2", 1, False, None, None),
    ("E2", "T4", 2, False, None, None), ("T4", "E3", 1, False, None, None),
    ("E3", "T5", 2, False, None, None), ("T5", "B4", 1, False, None, None),
    ("B4", "U3", 1, True, "E3", "S3"), ("S3", "D3", 1, False, None, None),
    ("D3", "U2", 1, True, "E2", "S2"), ("S2", "D2", 1, False, None, None),
    ("D2", "U1", 1, True, "E1", "S1"), ("S1", "D1", 1, False, None, None),
    ("D1", "U0", 1, True, "E0", "S0"), ("S0", "D0", 1, False, None, None),
]
HEAD_C = 16
# depth integral: source tensor, tensor it is appended to, channels, scale
SCAN_SRC, SCAN_DST, SCAN_C, SCAN_SCALE = "E0", "S0", 8, 1.0 / 16.0


def depth_sum_above(p):
    """Exclusive running sum over rows (axis 1): out[:, y] = sum_{v < y} p[:, v]."""
    out = np.zeros_like(p)
    out[:, 1:] = np.cumsum(p, axis=1)[:, :-1]
    return out


def depth_sum_below(g):
    """Adjoint of depth_sum_above: out[:, v] = sum_{y > v} g[:, y]."""
    out = np.zeros_like(g)
    out[:, :-1] = np.cumsum(g[:, ::-1], axis=1)[:, ::-1][:, 1:]
    return out


def param_layout():
    """[(name, offset, shape)] of the flat parameter vector."""
    out, off = [], 0
    for i, (src, dst, *_rest) in enumerate(LAYERS):
        ci, co = TENSORS[src][0], TENSORS[dst][0]
        out.append((f"w{i}", off, (co, 3, 3, ci)))
        off += co * 9 * ci
        out.append((f"b{i}", off, (co,)))
        off += co
    cs = TENSORS[SCAN_SRC][0]
    out.append(("wp", off, (SCAN_C, cs)))
    off += SCAN_C * cs
    out.append(("bp", off, (SCAN_C,)))
    off += SCAN_C
    out.append(("head_w", off, (HEAD_C,)))
    off += HEAD_C
    out.append(("head_b", off, (1,)))
    off += 1
    return out, off


def unflatten(flat):
    layout, n = param_layout()
    assert flat.size == n, (flat.size, n)
    return {name: np.asarray(flat[o:o + int(np.prod(shape))], dtype=np.float64).reshape(shape)
            for name, o, shape in layout}


def flatten(d):
    layout, n = param_layout()
    out = np.zeros(n)
    for name, o, shape in layout:
        out[o:o + int(np.prod(shape))] = d[name].ravel()
    return out


def forward(params, x, rounding=True):
    """params: dict (FP32 masters); x: NHWC input (8 channels).  Returns
    (activations dict, yhat [N,H,W])."""
    q = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    act = {"X": q(x)}
    for i, (src, dst, stride, up, skip, dst2) in enumerate(LAYERS):
        y = conv_forward(act[src], q(params[f"w{i}"]), params[f"b{i}"], stride=stride, pad=1, up=up, relu=True)
        act[dst] = q(y)
        if skip is not None:
            act[dst2] = q(act[dst] + act[skip])
            if dst2 == SCAN_DST:
                p = act[SCAN_SRC] @ q(params["wp"]).T + params["bp"]
                act[dst2] = np.concatenate([act[dst2], q(SCAN_SCALE * depth_sum_above(p))], axis=-1)
    yhat = act["D0"] @ q(params["head_w"]) + params["head_b"][0]
    return act, yhat


def l1_loss(yhat, y):
    return float(np.abs(yhat - y).mean())


def backward(params, act, yhat, y, rounding=True, extra_gy=None):
    """Gradients of the L1 loss (mean |yhat - y|) w.r.t. every parameter;
    extra_gy (optional, like yhat) is a further loss term's gradient at yhat
    (the adversarial term of the CT surrogate)."""
    q = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    P = yhat.size
    gy = np.sign(yhat - y) / P
    if extra_gy is not None:
        gy = gy + extra_gy
    grads = {"head_w": np.einsum("nhwc,nhw->c", act["D0"], gy), "head_b": np.array([gy.sum()])}
    g = {"D0": gy[..., None] * q(params["head_w"])[None, None, None, :]}
    for i in range(len(LAYERS) - 1, -1, -1):
        src, dst, stride, up, skip, dst2 = LAYERS[i]
        gout = g[dst2] if dst2 is not None else g[dst]
        if dst2 == SCAN_DST:
            # split the appended depth-integral channels off and back-propagate them
            gout, ga = gout[..., :-SCAN_C], gout[..., -SCAN_C:]
            dp = q(SCAN_SCALE * depth_sum_below(ga))
            grads["wp"] = np.einsum("nhwk,nhwc->kc", dp, act[SCAN_SRC])
            grads["bp"] = dp.sum(axis=(0, 1, 2))
            gs = dp @ q(params["wp"])
            g[SCAN_SRC] = g[SCAN_SRC] + gs if SCAN_SRC in g else gs
        dpre = q(gout * (act[dst] > 0))
        if skip is not None:
            g[skip] = g[skip] + gout if skip in g else gout.copy()
        dw, db = conv_backward_weight(act[src], dpre, k=3, stride=stride, pad=1, up=up)
        grads[f"w{i}"], grads[f"b{i}"] = dw, db
        if i > 0:
            dx = conv_backward_data(dpre, q(params[f"w{i}"]), act[src].shape, stride=stride, pad=1, up=up)
            g[src] = g[src] + dx if src in g else dx
    return grads


def loss_and_grads(flat_params, x, y, rounding=True):
    params = unflatten(flat_params)
    act, yhat = forward(params, x, rounding)
    return l1_loss(yhat, y), flatten(backward(params, act, yhat, y, rounding)), yhat


def psnr(yhat, y):
    """PSNR (peak 1) of clamp(yhat, 0, 1) against y."""
    mse = float(np.mean((np.clip(yhat, 0.0, 1.0) - y) ** 2))
    return 200.0 if mse == 0 else -10.0 * np.log10(mse)


def adam_update(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015) on FP64 copies; returns (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# CT-conditioned input (the learning-based simulator translates CT slices,
# Sec. 4 "Ultrasound simulation"; readings):
#   channel 0  nearest-voxel HU of the pixel (air, -1000 HU, outside the
#              volume) after histogram matching to a reference: the frame's
#              bins b = clip(HU + 1024, 0, 4095) map to the smallest reference
#              bin r with refC[r] * n_src >= srcC[b] * n_ref (C: inclusive
#              cumulative counts; exact integers), value (r - 1024) / 1000
#   channel 1  N0 of the voxel's noise draw (Box-Muller of its Philox words,
#              not gated); 0 outside
#   channel 2  N1 as the quantised normal Q[w2 >> 20] * 2^-20; 0 outside
#   channel 3  depth (y + 0.5) / H
# all bf16; channels 4..7 zero.

CT_BINS = 4096


def ct_bins(vol, probe, pose):
    """Histogram bins of the frame's nearest-voxel HU, [H][W] int64."""
    import oracle as _or
    o = _or.simulate_env(vol, _unit_table(vol), probe, pose, planes=("voxel",))
    vox = o["voxel"]
    hu = np.full(vox.shape, -1000, dtype=np.int64)
    inside = vox >= 0
    hu[inside] = np.asarray(vol.ct).ravel()[vox[inside]].astype(np.int64)
    return np.clip(hu + 1024, 0, CT_BINS - 1)


def _unit_table(vol):
    n = int(np.asarray(vol.labels).max()) + 1
    t = np.zeros((max(n, 1), 5), dtype=np.float32)
    t[:, 0] = 1.0
    return t


def ct_histogram(bins) -> np.ndarray:
    return np.bincount(np.asarray(bins).ravel(), minlength=CT_BINS).astype(np.int64)


def histogram_match_lut(src_hist, ref_hist) -> np.ndarray:
    """Bin map of histogram specification: lut[b] = smallest r with
    refC[r] * n_src >= srcC[b] * n_ref (exact in int64)."""
    sc = np.cumsum(np.asarray(src_hist, dtype=np.int64))
    rc = np.cumsum(np.asarray(ref_hist, dtype=np.int64))
    ns, nr = int(sc[-1]), int(rc[-1])
    return np.searchsorted(rc * ns, sc * nr, side="left").astype(np.int64)


def ct_input(vol, probe, pose, ref_hist) -> np.ndarray:
    """The 8-channel bf16 input of one frame (values as float64), [H][W][8]."""
    import oracle as _or
    o = _or.simulate_env(vol, _unit_table(vol), probe, pose, planes=("voxel", "philox"))
    vox, w = o["voxel"], o["philox"].astype(np.uint64)
    bins = ct_bins(vol, probe, pose)
    lut = histogram_match_lut(ct_histogram(bins), ref_hist)
    x = np.zeros(vox.shape + (8,))
    ct = (lut[bins] - 1024).astype(np.float32) / np.float32(1000.0)
    x[..., 0] = bf16_round(ct)
    inside = vox >= 0
    u0 = (2.0 * (w[..., 0] >> 9).astype(np.float64) + 1.0) / 16777216.0
    u1 = (2.0 * (w[..., 1] >> 9).astype(np.float64) + 1.0) / 16777216.0
    n0 = np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * np.pi * u1)
    q = _or.quantised_normal_table()
    n1 = q[(w[..., 2] >> 20).astype(np.int64)].astype(np.float64) * 2.0 ** -20
    x[..., 1] = np.where(inside, bf16_round(n0), 0.0)
    x[..., 2] = np.where(inside, bf16_round(n1), 0.0)
    H = probe.H
    x[..., 3] = bf16_round(((np.arange(H) + 0.5) / H)[:, None] * np.ones(vox.shape[1]))
    return x


# ---------------------------------------------------------------------------
# Adversarial term of the CT-conditioned surrogate (App. B.2: the pix2pix
# objective, L1 with weight 1 plus a GAN term with weight 0.01; pix2pix's
# discriminator judges patches of the image together with its input).
# Readings: a conditional patch discriminator of five 3x3 convs (pad 1),
#   8 -> 32 (stride 2), 32 -> 64 (2), 64 -> 128 (2), 128 -> 128 (1), 128 -> 8 (1),
# leaky ReLU (slope 0.2 in FP32) after the first four, no normalisation; the
# patch logit is channel 0 of the last conv (its other channels start at zero
# and receive no gradient).  Its input is the generator's input with channel
# 4 replaced by the image (bf16) and channels 5..7 zero.  Losses are the
# binary cross-entropy on logits l, softplus(-l) for "real" and softplus(l)
# for "fake", averaged over patches:
#   discriminator  L_D   = (mean_real softplus(-l) + mean_fake softplus(l)) / 2
#   generator      L_adv = mean softplus(-l(x, yhat))  (the non-saturating form)
# and one step runs in pix2pix's order: G forward, D update on the real pair
# (x, y) and the fake pair (x, yhat), then the G update on L1 + w L_adv with
# the updated D.

DISC_LAYERS = [(8, 32, 2), (32, 64, 2), (64, 128, 2), (128, 128, 1), (128, 8, 1)]   # (Ci, Co, stride)
LEAKY_SLOPE = float(np.float32(0.2))
DISC_IMAGE_C = 4


def disc_layout():
    """[(name, offset, shape)] of the discriminator's flat parameter vector."""
    out, off = [], 0
    for i, (ci, co, _st) in enumerate(DISC_LAYERS):
        out.append((f"dw{i}", off, (co, 3, 3, ci)))
        off += co * 9 * ci
        out.append((f"db{i}", off, (co,)))
        off += co
    return out, off


def disc_unflatten(flat):
    layout, n = disc_layout()
    assert flat.size == n, (flat.size, n)
    return {name: np.asarray(flat[o:o + int(np.prod(shape))], dtype=np.float64).reshape(shape)
            for name, o, shape in layout}


def disc_flatten(d):
    layout, n = disc_layout()
    out = np.zeros(n)
    for name, o, shape in layout:
        out[o:o + int(np.prod(shape))] = d[name].ravel()
    return out


def leaky_relu(a):
    a = np.asarray(a, dtype=np.float64)
    return np.where(a > 0, a, LEAKY_SLOPE * a)


def disc_input(x, img, rounding=True):
    """Discriminator input: x's channels 0..3, the image (bf16) in channel 4."""
    z = np.zeros(x.shape[:3] + (8,))
    z[..., :DISC_IMAGE_C] = x[..., :DISC_IMAGE_C]
    z[..., DISC_IMAGE_C] = bf16_round(img) if rounding else img
    return z


def disc_forward(dp, z, rounding=True):
    """Returns (activations [z, a1, .., a4], logits [N, H/8, W/8])."""
    q = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    act = [q(z)]
    last = len(DISC_LAYERS) - 1
    for i, (_ci, _co, st) in enumerate(DISC_LAYERS):
        y = conv_forward(act[-1], q(dp[f"dw{i}"]), dp[f"db{i}"], stride=st, pad=1)
        if i < last:
            act.append(q(leaky_relu(y)))
        else:
            logits = y[..., 0]
    return act, logits


def disc_backward(dp, act, dlogits, rounding=True, weights=True):
    """Back-propagates dlogits (gradient at the logits) through the
    discriminator: (parameter gradients or None, gradient at its input z)."""
    q = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    last = len(DISC_LAYERS) - 1
    g = np.zeros(dlogits.shape + (DISC_LAYERS[last][1],))
    g[..., 0] = dlogits
    grads = {} if weights else None
    for i in range(last, -1, -1):
        _ci, _co, st = DISC_LAYERS[i]
        dpre = q(g) if i == last else q(g * np.where(act[i + 1] > 0, 1.0, LEAKY_SLOPE))
        if weights:
            grads[f"dw{i}"], grads[f"db{i}"] = conv_backward_weight(act[i], dpre, k=3, stride=st, pad=1)
        g = conv_backward_data(dpre, q(dp[f"dw{i}"]), act[i].shape, stride=st, pad=1)
    return grads, g


def softplus(a):
    """log(1 + exp(a)), stable for large |a|."""
    a = np.asarray(a, dtype=np.float64)
    return np.maximum(a, 0.0) + np.log1p(np.exp(-np.abs(a)))


def sigmoid(a):
    a = np.asarray(a, dtype=np.float64)
    e = np.exp(-np.abs(a))
    return np.where(a >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def bce_logits(l, label):
    """Per-patch binary cross-entropy of logits l against label 1 or 0, and its
    derivative sigmoid(l) - label."""
    return (softplus(-l) if label else softplus(l)), sigmoid(l) - float(label)


def gan_train_step(gflat, dflat, x, y, adv_weight, lr, d_m=None, d_v=None, d_step=1, rounding=True):
    """One step of the CT surrogate with the adversarial term (order above).
    Returns a dict: yhat, l1, loss_d, loss_adv, d_grads and g_grads (flat),
    d_new (flat discriminator after its Adam step)."""
    gp, dp = unflatten(gflat), disc_unflatten(dflat)
    act, yhat = forward(gp, x, rounding)
    # discriminator step on the real and the fake pair
    act_r, l_r = disc_forward(dp, disc_input(x, y, rounding), rounding)
    act_f, l_f = disc_forward(dp, disc_input(x, yhat, rounding), rounding)
    (sr, gr), (sf, gf) = bce_logits(l_r, 1), bce_logits(l_f, 0)
    loss_d = 0.5 * (sr.mean() + sf.mean())
    dg_r, _ = disc_backward(dp, act_r, 0.5 * gr / l_r.size, rounding)
    dg_f, _ = disc_backward(dp, act_f, 0.5 * gf / l_f.size, rounding)
    d_grads = disc_flatten({k: dg_r[k] + dg_f[k] for k in dg_r})
    d_m = np.zeros_like(d_grads) if d_m is None else d_m
    d_v = np.zeros_like(d_grads) if d_v is None else d_v
    d_new, _m, _v = adam_update(np.asarray(dflat, dtype=np.float64), d_grads, d_m, d_v, d_step, lr)
    # generator's adversarial gradient through the updated discriminator
    dp2 = disc_unflatten(d_new)
    act_g, l_g = disc_forward(dp2, disc_input(x, yhat, rounding), rounding)
    sg, gg = bce_logits(l_g, 1)
    _, dz = disc_backward(dp2, act_g, adv_weight * gg / l_g.size, rounding, weights=False)
    g_grads = flatten(backward(gp, act, yhat, y, rounding, extra_gy=dz[..., DISC_IMAGE_C]))
    return dict(yhat=yhat, l1=l1_loss(yhat, y), loss_d=float(loss_d), loss_adv=float(sg.mean()),
                d_grads=d_grads, g_grads=g_grads, d_new=d_new)
