"""Batched persistent path (planes from device poses, work queue, HIP graph
replay, autotuner) vs the single-call path and the FP64 oracle (GPU)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth
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


@pytest.fixture(scope="module")
def uneven():
    """256 envs over 8 label volumes from 160^3 to 320x256x384, W in
    [64, 256], H in [128, 512]."""
    return synth.batched_workload(seed=0)


def batch_frames(sess, wl, vids, out=None, plan=None, steps=1, poses=None):
    from paper_2507_01152_amd import sonosim as sg
    offs, total = wl.out_offsets()
    if plan is None:
        plan = sg.sg_batch_plan_create(sess.ctx, vids, wl.probes, offs)
    sg.sg_batch_set_poses(sess.ctx, plan, wl.poses if poses is None else poses)
    if out is None:
        out = torch.full((total,), -7.0, dtype=torch.float32, device=sess.device)
    for _ in range(steps):
        sg.sg_batch_step(sess.ctx, plan, out)
    assert sg.sg_batch_status(sess.ctx, plan) == 0
    return out, plan


def test_batch_equals_single_call_bit_exact(sess, uneven):
    from paper_2507_01152_amd import sonosim as sg
    vids = sess.load(uneven)
    ref, _, _ = sess.simulate(uneven, vids)
    out, plan = batch_frames(sess, uneven, vids)
    torch.cuda.synchronize()
    assert torch.equal(ref, out)
    # graph replays are deterministic
    out2, _ = batch_frames(sess, uneven, vids, plan=plan, steps=3)
    assert torch.equal(out, out2)
    sg.sg_batch_plan_destroy(sess.ctx, plan)


def test_batch_256_envs_vs_oracle(sess, uneven):
    from paper_2507_01152_amd.session import split_frames
    vids = sess.load(uneven)
    out, plan = batch_frames(sess, uneven, vids)
    Y = split_frames(out.cpu().numpy(), uneven)

    def one(e):
        o = oracle.simulate_env(uneven.volumes[uneven.vol_ids[e]], uneven.table, uneven.probes[e],
                                uneven.poses[e], planes=("I", "A", "Y"))
        check_env({"Y": Y[e]}, o, uneven.probes[e], f"batched env {e}")
        return float(o["Y"].mean())

    with ThreadPoolExecutor(max_workers=16) as ex:
        means = list(ex.map(one, range(uneven.n_envs)))
    assert np.mean(means) > 0.02


def test_batch_mixing_window_and_wide_tiles(sess):
    """One batch whose PSF tiles take both the register-window path (lateral
    radius <= 8) and the per-pixel tap loop (up to 32 px), in every launch
    shape: bit-identical to single calls and within the oracle's bars."""
    from paper_2507_01152_amd import sonosim as sg
    from paper_2507_01152_amd.session import split_frames
    from synth import Probe, Workload
    base = synth.ellipsoid_workload(seed=13, n_envs=6, W=64, H=64)
    widths = [64, 300, 520, 1024, 90, 700]
    heights = [96, 64, 40, 33, 128, 70]
    psfs = [0.01, 0.01, 0.01, 0.0104, 0.01, 0.01]
    probes = [Probe(W=w, H=h, dx=0.06, dy=0.3, psf=f) for w, h, f in zip(widths, heights, psfs)]
    wl = Workload(base.volumes, base.vol_ids, probes, base.poses, base.table)
    vids = sess.load(wl)
    offs, total = wl.out_offsets()
    single = torch.zeros(total, dtype=torch.float32, device=sess.device)
    sg.sg_simulate(sess.ctx, vids, wl.probes, wl.poses, single, offs)
    plan = sg.sg_batch_plan_create(sess.ctx, vids, wl.probes, offs)
    for spw, tx in ((4, 16), (8, 32), (16, 64)):
        sg.sg_batch_set_config(sess.ctx, plan, spw, tx, 1)
        out, _ = batch_frames(sess, wl, vids, plan=plan)
        torch.cuda.synchronize()
        assert torch.equal(out, single), (spw, tx)
    Y = split_frames(single.cpu().numpy(), wl)
    for e in range(wl.n_envs):
        o = oracle.simulate_env(wl.volumes[wl.vol_ids[e]], wl.table, wl.probes[e], wl.poses[e], planes=("I", "A", "Y"))
        check_env({"Y": Y[e]}, o, wl.probes[e], f"wide batch env {e}")
    sg.sg_batch_plan_destroy(sess.ctx, plan)


def test_env_order_invariance(sess, uneven):
    """Permuting the environments (and their output slots) permutes frames."""
    from paper_2507_01152_amd.session import split_frames
    vids = sess.load(uneven)
    out, _ = batch_frames(sess, uneven, vids)
    perm = np.random.default_rng(1).permutation(uneven.n_envs)
    wl2 = synth.Workload(uneven.volumes, uneven.vol_ids[perm], [uneven.probes[i] for i in perm],
                         uneven.poses[perm], uneven.table)
    vids2 = vids[perm]
    out2, _ = batch_frames(sess, wl2, vids2)
    a = split_frames(out.cpu().numpy(), uneven)
    b = split_frames(out2.cpu().numpy(), wl2)
    for j, i in enumerate(perm):
        assert np.array_equal(a[i], b[j])


def test_autotune_keeps_frames_bit_identical(sess, uneven, tmp_path):
    from paper_2507_01152_amd import sonosim as sg
    vids = sess.load(uneven)
    out, plan = batch_frames(sess, uneven, vids)
    cache = str(tmp_path / "tune.jsonl")
    sg.sg_autotune(sess.ctx, plan, cache)
    spw, tx, ty, chunks = sg.sg_batch_config(sess.ctx, plan)
    assert spw in (4, 8, 16) and tx in (16, 32, 64) and ty == 64 and 1 <= chunks <= 4
    out2, _ = batch_frames(sess, uneven, vids, plan=plan)
    assert torch.equal(out, out2)
    text = open(cache).read()
    assert '"spw"' in text and "|n256|" in text
    # a second plan of the same shape reads the cache instead of timing
    out3, plan2 = batch_frames(sess, uneven, vids)
    sg.sg_autotune(sess.ctx, plan2, cache)
    assert sg.sg_batch_config(sess.ctx, plan2) == (spw, tx, ty, chunks)
    assert open(cache).read() == text
    ms_ray, ms_psf = sg.sg_batch_step_profiled(sess.ctx, plan2, out3)
    assert ms_ray > 0 and ms_psf > 0 and torch.equal(out, out3)


@pytest.mark.parametrize("spw,tx,chunks", [(4, 16, 1), (16, 64, 1), (8, 32, 2), (8, 64, 3), (4, 32, 4)])
def test_every_launch_shape_gives_identical_frames(sess, uneven, spw, tx, chunks):
    """Explicit launch shapes, including the chunked pipeline (PSF kernel of
    one env group beside the ray kernel of the next on a second stream), give
    the default shape's frames bit for bit, eagerly and through the graph."""
    from paper_2507_01152_amd import sonosim as sg
    vids = sess.load(uneven)
    ref, _ = batch_frames(sess, uneven, vids)
    out, plan = batch_frames(sess, uneven, vids)
    sg.sg_batch_set_config(sess.ctx, plan, spw, tx, chunks)
    assert sg.sg_batch_config(sess.ctx, plan) == (spw, tx, 64, chunks)
    for _ in range(3):   # graph replays
        out.fill_(-1.0)
        sg.sg_batch_step(sess.ctx, plan, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
    out.fill_(-1.0)
    ms_ray, ms_psf = sg.sg_batch_step_profiled(sess.ctx, plan, out)
    assert ms_ray > 0 and ms_psf > 0 and torch.equal(out, ref)
    assert sg.sg_batch_status(sess.ctx, plan) == 0


def test_set_config_rejects_bad_shapes(sess, uneven):
    from paper_2507_01152_amd import sonosim as sg
    vids = sess.load(uneven)
    _, plan = batch_frames(sess, uneven, vids)
    for bad in [(5, 32, 1), (8, 48, 1), (8, 32, 0), (8, 32, 5)]:
        with pytest.raises(sg.SonosimError):
            sg.sg_batch_set_config(sess.ctx, plan, *bad)


def test_volumetric_batch_equals_single_call_and_counts_envs(sess):
    """A plan of volumetric probes (5 planes each) gives the single-call
    frames bit for bit; a rejected pose zeroes all of its env's planes and
    counts once."""
    from paper_2507_01152_amd import sonosim as sg
    from paper_2507_01152_amd.session import split_frames
    wl = synth.volumetric_workload(seed=1, n_envs=6, n_vols=2)
    vids = sess.load(wl)
    one, offs, _ = sess.simulate(wl, vids)
    out, plan = batch_frames(sess, wl, vids)
    assert torch.equal(one, out)
    poses = wl.poses.copy()
    poses[4, 3] = 1e12
    sg.sg_batch_set_poses(sess.ctx, plan, poses)
    sg.sg_batch_step(sess.ctx, plan, out)
    assert sg.sg_batch_status(sess.ctx, plan) == 1
    frames = split_frames(out.cpu().numpy(), wl)
    assert frames[4].shape == (5, 50, 37) and not frames[4].any()
    ref = split_frames(one.cpu().numpy(), wl)
    for e in (0, 1, 2, 3, 5):
        assert np.array_equal(frames[e], ref[e])


def test_out_of_range_pose_gives_zero_frame_and_status(sess):
    from paper_2507_01152_amd import sonosim as sg
    wl = synth.ellipsoid_workload(seed=3, n_envs=3)
    vids = sess.load(wl)
    offs, total = wl.out_offsets()
    plan = sg.sg_batch_plan_create(sess.ctx, vids, wl.probes, offs)
    poses = wl.poses.copy()
    poses[1, 7] = 1e12
    poses[2, 0] = np.nan
    sg.sg_batch_set_poses(sess.ctx, plan, poses)
    out = torch.full((total,), -1.0, dtype=torch.float32, device=sess.device)
    sg.sg_batch_step(sess.ctx, plan, out)
    assert sg.sg_batch_status(sess.ctx, plan) == 2
    n = wl.probes[0].W * wl.probes[0].H
    y = out.cpu().numpy()
    assert (y[n:] == 0).all() and (y[:n] >= 0).all() and y[:n].max() > 0
    ref, _, _ = sess.simulate(synth.Workload(wl.volumes[:1], np.zeros(1, np.int32), wl.probes[:1],
                                             wl.poses[:1], wl.table), vids[:1])
    assert torch.equal(ref, out[:n])


@pytest.mark.parametrize("chunks", [1, 3])
def test_poses_changed_between_graph_replays(sess, chunks):
    """Every replay of one captured plan takes its planes from the poses then
    in the device buffer, and leaves its work counters ready for the next:
    poses A, then B (another set, one env out of range), then A again, each
    step bit-identical to the single-call path on the same poses."""
    from paper_2507_01152_amd import sonosim as sg
    wl = synth.ellipsoid_workload(seed=11, n_envs=6)
    wl_b = synth.ellipsoid_workload(seed=12, n_envs=6)
    vids = sess.load(wl)
    offs, total = wl.out_offsets()
    plan = sg.sg_batch_plan_create(sess.ctx, vids, wl.probes, offs)
    sg.sg_batch_set_config(sess.ctx, plan, 8, 32, chunks)
    poses_b = wl_b.poses.copy()
    poses_b[4, 3] = 1e12
    out = torch.full((total,), -7.0, dtype=torch.float32, device=sess.device)

    n4 = wl.probes[4].W * wl.probes[4].H
    lo, hi = int(offs[4]), int(offs[4]) + n4

    def single(poses):
        # the single call rejects an out-of-range pose outright: env 4 takes
        # an in-range one there and is compared separately
        p = poses.copy()
        p[4] = wl.poses[4]
        ref, _, _ = sess.simulate(synth.Workload(wl.volumes, wl.vol_ids, wl.probes, p, wl.table), vids)
        return ref

    for poses, n_bad in ((wl.poses, 0), (poses_b, 1), (wl.poses, 0)):
        sg.sg_batch_set_poses(sess.ctx, plan, poses)
        sg.sg_batch_step(sess.ctx, plan, out)
        assert sg.sg_batch_status(sess.ctx, plan) == n_bad
        ref = single(poses)
        torch.cuda.synchronize()
        assert torch.equal(out[:lo], ref[:lo]) and torch.equal(out[hi:], ref[hi:])
        if n_bad:
            assert (out[lo:hi] == 0).all()
        else:
            assert torch.equal(out[lo:hi], ref[lo:hi]) and out[lo:hi].max() > 0
    sg.sg_batch_plan_destroy(sess.ctx, plan)


def _plan_at_timed_shape(sess, wl, vids):
    """Plan of the workload at the launch shape the benchmark times (16
    scanlines per ray item, 64-wide PSF tiles, one chunk), stepped once."""
    from paper_2507_01152_amd import sonosim as sg
    offs, total = wl.out_offsets()
    out = torch.full((total,), -7.0, dtype=torch.float32, device=sess.device)
    plan = sg.sg_batch_plan_create(sess.ctx, vids, wl.probes, offs)
    sg.sg_batch_set_poses(sess.ctx, plan, wl.poses)
    sg.sg_batch_set_config(sess.ctx, plan, 16, 64, 1)
    sg.sg_batch_step(sess.ctx, plan, out)
    torch.cuda.synchronize()
    assert sg.sg_batch_status(sess.ctx, plan) == 0
    return out, plan


def _sampled_vs_oracle(wl, out, env_ids, name):
    from paper_2507_01152_amd.session import split_frames
    Y = split_frames(out.cpu().numpy(), wl)

    def one(e):
        o = oracle.simulate_env(wl.volumes[wl.vol_ids[e]], wl.table, wl.probes[e], wl.poses[e],
                                planes=("I", "A", "Y"))
        check_env({"Y": Y[e]}, o, wl.probes[e], f"{name} env {e}")
        return float(o["Y"].mean())

    with ThreadPoolExecutor(max_workers=16) as ex:
        return list(ex.map(one, env_ids))


def test_multiscale_batch_at_the_timed_shape_vs_oracle(sess, uneven):
    """The benchmark's multi-scale batch (the 256 uneven envs with S = 3 noise
    scales) at the timed launch shape: every 16th env against the oracle."""
    import dataclasses
    from paper_2507_01152_amd import sonosim as sg
    ms = dataclasses.replace(uneven, volumes=[dataclasses.replace(v, noise_scales=3) for v in uneven.volumes])
    vids = sess.load(ms)
    out, plan = _plan_at_timed_shape(sess, ms, vids)
    means = _sampled_vs_oracle(ms, out, range(0, ms.n_envs, 16), "S=3 batch")
    assert np.mean(means) > 0.02
    sg.sg_batch_plan_destroy(sess.ctx, plan)


def test_volumetric_batch_at_the_timed_shape_vs_oracle(sess):
    """The benchmark's volumetric batch (256 envs of 50 x 37 x 5 at 2 x 2 x 10
    mm) at the timed launch shape: every plane of every 16th env against the
    oracle."""
    from paper_2507_01152_amd import sonosim as sg
    vw = synth.volumetric_workload(seed=0)
    vids = sess.load(vw)
    out, plan = _plan_at_timed_shape(sess, vw, vids)
    means = _sampled_vs_oracle(vw, out, range(0, vw.n_envs, 16), "volumetric batch")
    assert np.mean(means) > 0.0
    sg.sg_batch_plan_destroy(sess.ctx, plan)
