"""Reconstruction observation of the bone-surface task (surface points with
misses, accumulated over steps, voxelised in the current probe frame)
through the C ABI vs the oracle (GPU)."""
import numpy as np
import pytest

import oracle
import synth
from synth import Probe

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


def _moved(poses, step):
    """Poses shifted along their own lateral axis by 3 mm per step and tilted."""
    out = poses.copy().reshape(-1, 3, 4)
    c, s = np.cos(0.05 * step), np.sin(0.05 * step)
    Ry = np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])
    for i in range(out.shape[0]):
        R = out[i, :, :3]
        out[i, :, 3] += R[:, 0] * (3.0 * step)
        out[i, :, :3] = R @ Ry
    return out.reshape(-1, 12)


def _workload():
    wl = synth.batched_workload(seed=4, n_envs=5, n_vols=2, W_range=(40, 120), H_range=(150, 300))
    wl.probes[3] = Probe(W=37, H=50, dx=2.0, dy=2.0, n_elev=5, elev=10.0)   # volumetric probe
    return wl


def test_recon_points_and_grids_match_oracle(sess):
    from paper_2507_01152_amd import sonosim as sg
    wl = _workload()
    vids = sess.load(wl)
    offs, total = wl.out_offsets()
    plan = sg.sg_batch_plan_create(sess.ctx, vids, wl.probes, offs)
    out = torch.empty(total, dtype=torch.float32, device=sess.device)
    rid = sg.sg_recon_create(sess.ctx, plan, 20000, None, 0.2, seed=77)
    steps = 4
    ref_pts = [[] for _ in range(wl.n_envs)]
    for st in range(steps):
        poses = _moved(wl.poses, st)
        sg.sg_batch_set_poses(sess.ctx, plan, poses)
        sg.sg_batch_step(sess.ctx, plan, out)
        sg.sg_recon_update(sess.ctx, rid, st)
        for e in range(wl.n_envs):
            ref_pts[e].append(oracle.recon_points(wl.volumes[wl.vol_ids[e]], wl.probes[e], poses[e], e, st, 77, 0.2))
    grids = torch.zeros(wl.n_envs * 40 ** 3, dtype=torch.uint8, device=sess.device)
    sg.sg_recon_observe(sess.ctx, rid, grids)
    stored, over = sg.sg_recon_counts(sess.ctx, rid, wl.n_envs)
    g = grids.cpu().numpy().reshape(wl.n_envs, 40, 40, 40)
    last = _moved(wl.poses, steps - 1)
    for e in range(wl.n_envs):
        ref = np.concatenate(ref_pts[e])
        assert stored[e] == ref.shape[0] and over[e] == 0
        got = sg.sg_recon_points(sess.ctx, rid, e, 20000)
        # order is unspecified: compare the sorted point sets bit for bit
        key = lambda a: a[np.lexsort(a.T[::-1])]
        assert np.array_equal(key(got), key(ref)), e
        assert np.array_equal(g[e], oracle.recon_observe(ref, last[e])), e
    assert stored.sum() > 100 and g.sum() > 50
    # reset of one env, then capacity overflow is counted
    sg.sg_recon_reset(sess.ctx, rid, 1)
    s2, _ = sg.sg_recon_counts(sess.ctx, rid, wl.n_envs)
    assert s2[1] == 0 and s2[0] == stored[0]
    sg.sg_recon_destroy(sess.ctx, rid)
    small = sg.sg_recon_create(sess.ctx, plan, 10, [3], 0.0, seed=1)
    sg.sg_recon_update(sess.ctx, small, 0)
    s3, o3 = sg.sg_recon_counts(sess.ctx, small, wl.n_envs)
    for e in range(wl.n_envs):
        n = oracle.recon_points(wl.volumes[wl.vol_ids[e]], wl.probes[e], last[e], e, 0, 1, 0.0).shape[0]
        assert s3[e] == min(n, 10) and o3[e] == max(0, n - 10)
    sg.sg_recon_destroy(sess.ctx, small)
    sg.sg_batch_plan_destroy(sess.ctx, plan)


def test_recon_rejects_bad_arguments(sess):
    from paper_2507_01152_amd import sonosim as sg
    wl = _workload()
    vids = sess.load(wl)
    offs, _ = wl.out_offsets()
    plan = sg.sg_batch_plan_create(sess.ctx, vids, wl.probes, offs)
    for args in [(plan + 1000, 10, None, 0.2), (plan, 0, None, 0.2), (plan, 10, None, 1.5)]:
        with pytest.raises(sg.SonosimError):
            sg.sg_recon_create(sess.ctx, *args)
    rid = sg.sg_recon_create(sess.ctx, plan, 10)
    sg.sg_batch_plan_destroy(sess.ctx, plan)
    with pytest.raises(sg.SonosimError):
        sg.sg_recon_update(sess.ctx, rid, 0)
    sg.sg_recon_destroy(sess.ctx, rid)


def test_recon_benchmark_batch_sampled_vs_oracle(sess):
    """The benchmark's reconstruction leg at full size: the 256 envs of the
    benchmark batch stepped once at the timed launch shape, then 20 updates
    (capacity 65536 points, 20 % drop, seed 1) and the 40^3 observation: the
    stored points and the grid of every 16th env against the oracle."""
    from paper_2507_01152_amd import sonosim as sg
    wl = synth.batched_workload(seed=0)
    n = wl.n_envs
    vids = sess.load(wl)
    offs, total = wl.out_offsets()
    plan = sg.sg_batch_plan_create(sess.ctx, vids, wl.probes, offs)
    sg.sg_batch_set_poses(sess.ctx, plan, wl.poses)
    sg.sg_batch_set_config(sess.ctx, plan, 16, 64, 1)
    out = torch.empty(total, dtype=torch.float32, device=sess.device)
    sg.sg_batch_step(sess.ctx, plan, out)
    rid = sg.sg_recon_create(sess.ctx, plan, 65536, None, 0.2, seed=1)
    for st in range(20):
        sg.sg_recon_update(sess.ctx, rid, st)
    grids = torch.zeros(n * 40 ** 3, dtype=torch.uint8, device=sess.device)
    sg.sg_recon_observe(sess.ctx, rid, grids)
    stored, over = sg.sg_recon_counts(sess.ctx, rid, n)
    g = grids.cpu().numpy().reshape(n, 40, 40, 40)
    key = lambda a: a[np.lexsort(a.T[::-1])]
    total_pts = 0
    for e in range(0, n, 16):
        ref = np.concatenate([oracle.recon_points(wl.volumes[wl.vol_ids[e]], wl.probes[e], wl.poses[e], e, st, 1, 0.2)
                              for st in range(20)])
        assert stored[e] == ref.shape[0] and over[e] == 0, e
        got = sg.sg_recon_points(sess.ctx, rid, e, 65536)
        assert np.array_equal(key(got), key(ref)), e
        assert np.array_equal(g[e], oracle.recon_observe(ref, wl.poses[e])), e
        total_pts += ref.shape[0]
    assert total_pts > 100
    sg.sg_recon_destroy(sess.ctx, rid)
    sg.sg_batch_plan_destroy(sess.ctx, plan)
