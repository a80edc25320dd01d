"""CT-conditioned surrogate through the C ABI vs the oracle (GPU): the pooled
reference histogram, the per-frame histogram specification and the
8-channel input, bit for bit where both sides decide in the same precision."""
import numpy as np
import pytest

import synth
from cases import axis_pose
from oracle import surrogate as so
from synth import Probe, Volume, Workload
from tolerance import check_env

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sess():
    from paper_2507_01152_amd.session import Session
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = Session(0)
    yield s
    s.close()


def _oracle_reference(wl, envs):
    h = np.zeros(so.CT_BINS, dtype=np.int64)
    for e in envs:
        h += so.ct_histogram(so.ct_bins(wl.volumes[wl.vol_ids[e]], wl.probes[e], wl.poses[e]))
    return h


def _check_inputs(x, wl, envs, ref):
    for i, e in enumerate(envs):
        o = so.ct_input(wl.volumes[wl.vol_ids[e]], wl.probes[e], wl.poses[e], ref)
        g = x[i]
        for c in (0, 2, 3, 4, 5, 6, 7):
            assert np.array_equal(g[..., c], o[..., c]), f"env {e} channel {c}"
        # N0: hardware log / sqrt / cos in FP32 vs FP64, then bf16: within one bf16 step
        assert np.array_equal(g[..., 1] == 0, o[..., 1] == 0)
        assert np.all(np.abs(g[..., 1] - o[..., 1]) <= 2.0 ** -7 * np.abs(o[..., 1]) + 1e-6), f"env {e} N0"


def _mixed_workload():
    """Spine CT phantom (96^3) at 64 x 128, plus a small CT volume whose HU
    reach both clamps of the bins and a pose that leaves the grid (air)."""
    wl = synth.spine_ct_workload(seed=4, n_envs=6, dims=(96, 96, 96), W=64, H=128)
    lab = np.ones((40, 24, 24), dtype=np.uint8)
    lab[25:] = 3
    rng = np.random.default_rng(8)
    ct = rng.integers(-1500, 4000, size=lab.shape).astype(np.int16)
    small = Volume(labels=lab, ct=ct, seed=12)
    poses = np.concatenate([wl.poses, axis_pose((12.0, 12.0, -20.0))[None], axis_pose((-10.0, 12.0, 5.0))[None]])
    probes = list(wl.probes) + [Probe(W=64, H=128, dx=0.5, dy=0.5), Probe(W=64, H=128, dx=0.5, dy=0.5)]
    return Workload([wl.volumes[0], small], np.array([0] * 6 + [1, 1], dtype=np.int32), probes, poses)


def test_ct_reference_and_input_parity(sess):
    from paper_2507_01152_amd import sonosim as sg
    wl = _mixed_workload()
    vids = sess.load(wl)
    H, W = 128, 64
    sid = sg.sg_surr_create_ct(sess.ctx, H, W, seed=1)
    ref_envs = [0, 1, 2, 6]
    hist = sg.sg_surr_set_ct_reference(sess.ctx, sid, vids[ref_envs], [wl.probes[e] for e in ref_envs],
                                       wl.poses[ref_envs])
    ref = _oracle_reference(wl, ref_envs)
    assert np.array_equal(hist, ref)
    assert hist.sum() == len(ref_envs) * H * W and hist[0] > 0 and hist[-1] > 0   # both clamps are hit
    envs = [3, 4, 5, 7]
    sg.sg_surr_train_step(sess.ctx, sid, vids[envs], [wl.probes[e] for e in envs], wl.poses[envs], 0.0)
    xin, tgt = sg.sg_surr_get_batch(sess.ctx, sid, len(envs), H, W)
    _check_inputs(so.bf16_bits_to_f64(xin), wl, envs, ref)
    # the physics targets (rendered by the CT ray instantiation without debug
    # planes) against the oracle's frames
    import oracle
    for i, e in enumerate(envs):
        o = oracle.simulate_env(wl.volumes[wl.vol_ids[e]], wl.table, wl.probes[e], wl.poses[e],
                                planes=("I", "A", "Y"))
        check_env({"Y": tgt[i]}, o, wl.probes[e], f"CT target env {e}")
    sg.sg_surr_destroy(sess.ctx, sid)


def test_ct_matching_against_itself_is_identity_on_used_bins(sess):
    """A frame matched to a reference equal to its own histogram keeps its HU."""
    from paper_2507_01152_amd import sonosim as sg
    wl = _mixed_workload()
    vids = sess.load(wl)
    H, W = 128, 64
    sid = sg.sg_surr_create_ct(sess.ctx, H, W, seed=2)
    sg.sg_surr_set_ct_reference(sess.ctx, sid, vids[[3]], [wl.probes[3]], wl.poses[[3]])
    sg.sg_surr_train_step(sess.ctx, sid, vids[[3]], [wl.probes[3]], wl.poses[[3]], 0.0)
    xin, _ = sg.sg_surr_get_batch(sess.ctx, sid, 1, H, W)
    b = so.ct_bins(wl.volumes[0], wl.probes[3], wl.poses[3])
    want = so.bf16_round((b - 1024).astype(np.float32) / np.float32(1000.0))
    assert np.array_equal(so.bf16_bits_to_f64(xin[0, ..., 0]), want)
    sg.sg_surr_destroy(sess.ctx, sid)


def test_ct_checkpoint_keeps_the_reference(sess, tmp_path):
    from paper_2507_01152_amd import sonosim as sg
    wl = _mixed_workload()
    vids = sess.load(wl)
    H, W = 128, 64
    sid = sg.sg_surr_create_ct(sess.ctx, H, W, seed=3)
    sg.sg_surr_set_ct_reference(sess.ctx, sid, vids[:3], wl.probes[:3], wl.poses[:3])
    sg.sg_surr_train_step(sess.ctx, sid, vids[3:5], wl.probes[3:5], wl.poses[3:5], 1e-3)
    path = str(tmp_path / "ct.ckpt")
    sg.sg_surr_save(sess.ctx, sid, path)
    sid2 = sg.sg_surr_create_ct(sess.ctx, H, W, seed=77)
    sg.sg_surr_load(sess.ctx, sid2, path)
    for s in (sid, sid2):
        sg.sg_surr_train_step(sess.ctx, s, vids[5:7], wl.probes[5:7], wl.poses[5:7], 1e-3)
    a = sg.sg_surr_get_batch(sess.ctx, sid, 2, H, W)
    b = sg.sg_surr_get_batch(sess.ctx, sid2, 2, H, W)
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(sg.sg_surr_get_params(sess.ctx, sid), sg.sg_surr_get_params(sess.ctx, sid2))
    # label-mode checkpoints do not load into a CT surrogate, nor the reverse
    plain = sg.sg_surr_create(sess.ctx, H, W, seed=3)
    with pytest.raises(sg.SonosimError):
        sg.sg_surr_load(sess.ctx, plain, path)
    for s in (sid, sid2, plain):
        sg.sg_surr_destroy(sess.ctx, s)


def test_ct_surrogate_errors(sess):
    from paper_2507_01152_amd import sonosim as sg
    wl = _mixed_workload()
    vids = sess.load(wl)
    H, W = 128, 64
    with pytest.raises(sg.SonosimError) as e:
        sg.sg_surr_create_ct(sess.ctx, H, W, seed=1, adv_weight=2.0)
    assert e.value.status == sg.SG_EINVAL
    sid = sg.sg_surr_create_ct(sess.ctx, H, W, seed=1)
    with pytest.raises(sg.SonosimError) as e:   # no reference yet
        sg.sg_surr_train_step(sess.ctx, sid, vids[:1], wl.probes[:1], wl.poses[:1], 0.0)
    assert e.value.status == sg.SG_ESTATE
    lab_only = synth.ellipsoid_workload(seed=1, n_envs=1, W=W, H=H)
    lv = sess.load(lab_only)
    with pytest.raises(sg.SonosimError) as e:   # a volume without CT
        sg.sg_surr_set_ct_reference(sess.ctx, sid, lv, lab_only.probes, lab_only.poses)
    assert e.value.status == sg.SG_EINVAL
    with pytest.raises(sg.SonosimError) as e:   # wrong frame size
        sg.sg_surr_set_ct_reference(sess.ctx, sid, vids[:1], [Probe(W=32, H=H)], wl.poses[:1])
    assert e.value.status == sg.SG_EINVAL
    plain = sg.sg_surr_create(sess.ctx, H, W, seed=1)
    with pytest.raises(sg.SonosimError) as e:
        sg.sg_surr_set_ct_reference(sess.ctx, plain, vids[:1], wl.probes[:1], wl.poses[:1])
    assert e.value.status == sg.SG_EINVAL
    sg.sg_surr_set_ct_reference(sess.ctx, sid, vids[:1], wl.probes[:1], wl.poses[:1])
    with pytest.raises(sg.SonosimError) as e:
        sg.sg_surr_train_step(sess.ctx, sid, lv, lab_only.probes, lab_only.poses, 0.0)
    assert e.value.status == sg.SG_EINVAL
    for s in (sid, plain):
        sg.sg_surr_destroy(sess.ctx, s)


# ---------------------------------------------------------------------------
# adversarial term: discriminator and generator gradients of one step


def _gan_problem(seed, n=4, H=128, W=64):
    """Seeded parameters of both networks and CT-style input pairs."""
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
    g[dict((nm, o) for nm, o, _ in layout)["head_b"]] = 0.2
    dl, nd = so.disc_layout()
    d = np.zeros(nd)
    for name, o, shape in dl:
        sz = int(np.prod(shape))
        if name.startswith("dw"):
            w = rng.standard_normal(shape) * np.sqrt(2.0 / np.prod(shape[1:]))
            if name == "dw4":
                w[1:] = 0.0   # the logit conv's unused channels
            d[o:o + sz] = w.ravel()
        else:
            d[o:o + sz] = rng.standard_normal(sz) * 0.02
            if name == "db4":
                d[o + 1:o + sz] = 0.0
    x = np.zeros((n, H, W, 8))
    x[..., 0] = so.bf16_round(rng.normal(0.1, 0.5, (n, H, W)))
    x[..., 1] = so.bf16_round(rng.standard_normal((n, H, W)))
    x[..., 2] = so.bf16_round(rng.standard_normal((n, H, W)))
    x[..., 3] = so.bf16_round((np.arange(H) + 0.5) / H)[None, :, None]
    y = np.clip(0.3 + 0.4 * np.tanh(x[..., 0]) + 0.1 * rng.standard_normal((n, H, W)), 0, 1).astype(np.float32)
    return g.astype(np.float32), d.astype(np.float32), x, y


def _per_layer(a, b, layout):
    out = []
    for name, o, shape in layout:
        sz = int(np.prod(shape))
        u, v = a[o:o + sz], b[o:o + sz]
        if not np.any(v):
            out.append((name, float(np.abs(u).max()), 1.0))
            continue
        err = np.linalg.norm(u - v) / np.linalg.norm(v)
        cos = float(u @ v) / max(np.linalg.norm(u) * np.linalg.norm(v), 1e-30)
        out.append((name, round(float(err), 5), round(cos, 6)))
    return out


def test_gan_step_gradients_match_oracle(sess):
    """One step at learning rate 0 (both Adam steps leave the weights, so the
    discriminator that judges the generator is the one differentiated):
    the losses, every discriminator layer's gradient and every generator
    layer's gradient of L1 + w L_adv against the oracle on the same seeded
    parameters and pairs.  bf16 flips of single activations give per-layer
    differences of about 1e-3 to 2e-2 in norm, as for the L1-only network;
    the discriminator's first layer, behind four bf16 layers of its own,
    has the most, so the batch is 8 frames (noise falls as one over the root
    of the pixel count).  The adversarial part alone (w = 1 minus w = 0) is
    compared too; as a difference of two noisy gradients it gets 5e-2."""
    from paper_2507_01152_amd import sonosim as sg
    n, H, W = 8, 128, 64
    gp, dp, x, y = _gan_problem(31, n, H, W)
    xin = torch.from_numpy(so.f64_to_bf16_bits(x).view(np.int16)).cuda()
    tgt = torch.from_numpy(y).cuda()
    grads = {}
    for w in (1.0, 0.0):
        sid = sg.sg_surr_create_ct(sess.ctx, H, W, seed=5, adv_weight=max(w, 1e-30))
        sg.sg_surr_set_params(sess.ctx, sid, gp)
        sg.sg_surr_disc_set_params(sess.ctx, sid, dp)
        loss = sg.sg_surr_train_pairs(sess.ctx, sid, xin, tgt, 0.0)
        ld, ladv = sg.sg_surr_gan_losses(sess.ctx, sid)
        grads[w] = (sg.sg_surr_get_grads(sess.ctx, sid).astype(np.float64),
                    sg.sg_surr_disc_get_grads(sess.ctx, sid).astype(np.float64), loss, ld, ladv)
        assert np.array_equal(sg.sg_surr_disc_get_params(sess.ctx, sid), dp)   # lr 0
        sg.sg_surr_destroy(sess.ctx, sid)
    ref = so.gan_train_step(gp.astype(np.float64), dp.astype(np.float64), x, y.astype(np.float64), 1.0, 0.0)
    ref0 = so.gan_train_step(gp.astype(np.float64), dp.astype(np.float64), x, y.astype(np.float64), 0.0, 0.0)
    g1, d1, loss, ld, ladv = grads[1.0]
    print("losses gpu", loss, ld, ladv, "oracle", ref["l1"], ref["loss_d"], ref["loss_adv"])
    assert abs(loss - ref["l1"]) <= 1e-3 * ref["l1"]
    assert abs(ld - ref["loss_d"]) <= 2e-3 * ref["loss_d"]
    assert abs(ladv - ref["loss_adv"]) <= 2e-3 * ref["loss_adv"]
    rep_d = _per_layer(d1, ref["d_grads"], so.disc_layout()[0])
    rep_g = _per_layer(g1, ref["g_grads"], so.param_layout()[0])
    adv_gpu, adv_ref = g1 - grads[0.0][0], ref["g_grads"] - ref0["g_grads"]
    rep_a = _per_layer(adv_gpu, adv_ref, so.param_layout()[0])
    print("disc", rep_d)
    print("gen", rep_g)
    print("adv part", rep_a)
    bad = [r for r in rep_d + rep_g if not (r[1] <= 2e-2 and r[2] >= 0.999)]
    assert not bad, bad
    bad = [r for r in rep_a if not (r[1] <= 5e-2 and r[2] >= 0.998)]
    assert not bad, bad
    # the logit conv's unused channels get no gradient
    o = dict((nm, off) for nm, off, _ in so.disc_layout()[0])["dw4"]
    assert not d1[o + 9 * 128:o + 8 * 9 * 128].any()


def test_gan_step_updates_in_pix2pix_order(sess, tmp_path):
    """At a positive rate both networks take Adam's first step on their own
    gradients, the generator's gradient is taken through the updated
    discriminator (it differs from the rate-0 one), and a checkpoint restores
    both networks bit for bit."""
    from paper_2507_01152_amd import sonosim as sg
    n, H, W = 2, 64, 64
    gp, dp, x, y = _gan_problem(32, n, H, W)
    xin = torch.from_numpy(so.f64_to_bf16_bits(x).view(np.int16)).cuda()
    tgt = torch.from_numpy(y).cuda()
    lr = 1e-3
    out = {}
    for rate in (0.0, lr):
        sid = sg.sg_surr_create_ct(sess.ctx, H, W, seed=6, adv_weight=0.01)
        sg.sg_surr_set_params(sess.ctx, sid, gp)
        sg.sg_surr_disc_set_params(sess.ctx, sid, dp)
        sg.sg_surr_train_pairs(sess.ctx, sid, xin, tgt, rate)
        out[rate] = [sg.sg_surr_get_grads(sess.ctx, sid).astype(np.float64),
                     sg.sg_surr_disc_get_grads(sess.ctx, sid).astype(np.float64),
                     sg.sg_surr_get_params(sess.ctx, sid).astype(np.float64),
                     sg.sg_surr_disc_get_params(sess.ctx, sid).astype(np.float64), sid]
    g, dg, p1, d1, sid = out[lr]
    assert np.allclose(d1, dp - lr * dg / (np.abs(dg) + 1e-8), rtol=1e-4, atol=1e-6 * lr)
    assert np.allclose(p1, gp - lr * g / (np.abs(g) + 1e-8), rtol=1e-4, atol=1e-6 * lr)
    assert np.array_equal(dg, out[0.0][1])           # the discriminator's gradient precedes its update
    assert not np.array_equal(g, out[0.0][0])        # the generator is judged by the updated one
    path = str(tmp_path / "gan.ckpt")
    sg.sg_surr_save(sess.ctx, sid, path)
    sid2 = sg.sg_surr_create_ct(sess.ctx, H, W, seed=99, adv_weight=0.01)
    sg.sg_surr_load(sess.ctx, sid2, path)
    for s in (sid, sid2):
        sg.sg_surr_train_pairs(sess.ctx, s, xin, tgt, lr)
    assert np.array_equal(sg.sg_surr_disc_get_params(sess.ctx, sid), sg.sg_surr_disc_get_params(sess.ctx, sid2))
    assert np.array_equal(sg.sg_surr_get_params(sess.ctx, sid), sg.sg_surr_get_params(sess.ctx, sid2))
    assert sg.sg_surr_gan_losses(sess.ctx, sid) == sg.sg_surr_gan_losses(sess.ctx, sid2)
    plain_ct = sg.sg_surr_create_ct(sess.ctx, H, W, seed=1)   # no discriminator: other checkpoint kind
    with pytest.raises(sg.SonosimError):
        sg.sg_surr_load(sess.ctx, plain_ct, path)
    with pytest.raises(sg.SonosimError):
        sg.sg_surr_gan_losses(sess.ctx, plain_ct)
    with pytest.raises(sg.SonosimError):   # frame size of the buffers
        sg.sg_surr_train_pairs(sess.ctx, sid, xin[:, :32].contiguous(), tgt[:, :32].contiguous(), lr)
    for s in (out[0.0][4], sid, sid2, plain_ct):
        sg.sg_surr_destroy(sess.ctx, s)


def test_ct_gan_training_gains_over_untrained(sess):
    """A short run of the CT surrogate with the adversarial term (weight
    0.01) on spine CT phantom pairs: on held-out phantoms its frames beat the
    untrained network's by a wide margin, and both adversarial losses stay
    finite and in the range a working discriminator gives (L_D < 2 log 2)."""
    from paper_2507_01152_amd import sonosim as sg
    from paper_2507_01152_amd.train_surrogate import CT_FRAME_H, CT_FRAME_W, CtPairSource, train_ct
    s2, sid, src, _step_s, last = train_ct(400, 16, 1e-3, adv_weight=0.01, n_train_vols=6, log=print)
    held = CtPairSource(s2, 2, seed0=9100)
    rng = np.random.default_rng(5)
    vids, probes, poses = held.batch(32, rng)
    out = torch.empty(32 * CT_FRAME_W * CT_FRAME_H, dtype=torch.float32, device=s2.device)
    psnr_net, _ = sg.sg_surr_infer(s2.ctx, sid, vids, probes, poses, out, list(range(32)), -np.inf, 1.0)
    fresh = sg.sg_surr_create_ct(s2.ctx, CT_FRAME_H, CT_FRAME_W, seed=1, adv_weight=0.01)
    sg.sg_surr_set_ct_reference(s2.ctx, fresh, *src.batch(16, np.random.default_rng(3)))
    psnr_init, _ = sg.sg_surr_infer(s2.ctx, fresh, vids, probes, poses, out, list(range(32)), -np.inf, 1.0)
    print(f"held-out PSNR: trained {np.mean(psnr_net):.2f} dB, untrained {np.mean(psnr_init):.2f} dB; {last}")
    assert np.mean(psnr_net) - np.mean(psnr_init) > 5.0
    assert np.isfinite(last["loss_d"]) and 0.0 < last["loss_d"] < 2 * np.log(2.0)
    assert np.isfinite(last["loss_adv"]) and last["loss_adv"] > 0.0
    s2.close()
