"""HIP physics path vs the FP64 oracle, through the C ABI (GPU)."""
import numpy as np
import pytest

import oracle
import synth
from cases import axis_pose, layered_volume, single_env, table_with
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


def run_gpu(sess, wl, debug=True):
    from paper_2507_01152_amd.session import split_frames
    vids = sess.load(wl)
    out, offs, dbg = sess.simulate(wl, vids, debug=debug)
    torch.cuda.synchronize()
    res = [dict(Y=y) for y in split_frames(out.cpu().numpy(), wl)]
    if debug:
        for k, t in dbg.items():
            per = 4 if k == "philox" else 1
            for e, a in enumerate(split_frames(t.cpu().numpy(), wl, per)):
                res[e][k] = a
    return res


def check_all(sess, wl, env_ids=None, name="", debug=True):
    g = run_gpu(sess, wl, debug=debug)
    ids = range(wl.n_envs) if env_ids is None else env_ids
    for e in ids:
        o = oracle.simulate_env(wl.volumes[wl.vol_ids[e]], wl.table, wl.probes[e], wl.poses[e],
                                planes=("label", "voxel", "philox", "E", "T", "I", "A", "Y"))
        check_env(g[e], o, wl.probes[e], f"{name} env {e}")
    return g


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_ellipsoid_64_cubed_parity(sess, seed):
    """64^3 label volume, 6 ellipsoids, 64 scanlines x 128 samples."""
    wl = synth.ellipsoid_workload(seed=seed, n_envs=4)
    g = check_all(sess, wl, name=f"seed{seed}")
    assert any((x["label"] == 3).any() for x in g)   # bone is hit somewhere


@pytest.mark.parametrize("W,H", [(1, 1), (1, 200), (37, 101), (64, 65), (200, 1), (130, 300), (3, 700)])
def test_ragged_and_degenerate_sizes(sess, W, H):
    wl = synth.ellipsoid_workload(seed=7, n_envs=2, W=W, H=H, dx=0.37, dy=0.29)
    check_all(sess, wl, name=f"{W}x{H}")


@pytest.mark.parametrize("W,H,psf", [(400, 64, 0.01), (300, 50, 0.0104), (1024, 40, 0.0104)])
def test_wide_frames_take_the_per_pixel_lateral_taps(sess, W, H, psf):
    """Lateral PSF radii above 8 px (frames wider than 266 px at 1 % of the
    width) take the PSF kernel's per-pixel tap loop instead of the register
    window; 1024 x 40 at 0.0104 gives the 32 px radius limit."""
    wl = synth.ellipsoid_workload(seed=9, n_envs=1, W=W, H=H, dx=0.06, dy=0.3)
    for p in wl.probes:
        p.psf = psf
    check_all(sess, wl, name=f"{W}x{H} psf {psf}")


def test_maximum_frame_1024_square(sess):
    """The largest frame (1024 x 1024): axial and lateral radii 31 px."""
    wl = synth.ellipsoid_workload(seed=10, n_envs=1, W=1024, H=1024, dx=0.06, dy=0.06)
    check_all(sess, wl, name="1024x1024", debug=False)


def test_plane_entirely_outside_volume(sess):
    vol = Volume(labels=np.ones((16, 16, 16), dtype=np.uint8), seed=4)
    wl = single_env(vol, Probe(W=20, H=40), axis_pose((-500.0, -500.0, -500.0)))
    g = check_all(sess, wl, name="outside")
    assert (g[0]["voxel"] == -1).all() and (g[0]["Y"] == 0).all()


@pytest.mark.parametrize("Zb", [np.inf, 0.0])
def test_total_reflection_at_bone(sess, Zb):
    table = table_with(Z_3=Zb)
    vol = layered_volume(64, 64, 64, [(0, 1), (15, 3)])
    wl = single_env(vol, Probe(W=15, H=120), axis_pose((32.0, 32.0, 0.0)), table)
    g = check_all(sess, wl, name=f"Zbone={Zb}")
    assert (g[0]["energy"][29:] == 0).all() and (g[0]["energy"][:29] > 0).all()


def test_deep_attenuation_down_to_the_energy_floor(sess):
    """1024 rows through strongly attenuating tissue: E falls to about
    2^-81 E0 at the bottom (3e-25 E0, above the 1e-30 E0 floor of the
    tolerance); the GPU's FP32 running sum of alpha (tree order within a
    chunk, compensated across 16 chunks) must keep E within 1e-4 E."""
    table = table_with(alpha_1=2.0, alpha_2=1.0)
    vol = layered_volume(16, 16, 80, [(0, 1), (30, 2), (45, 1)])
    wl = single_env(vol, Probe(W=3, H=1024, dx=1.0, dy=0.0625), axis_pose((8.0, 8.0, 0.0)), table)
    g = check_all(sess, wl, name="deep")
    E = g[0]["energy"]
    assert (E[-1] > 1e-26).all() and (E[-1] < 1e-24).all()


@pytest.mark.parametrize("scales", [2, 3, 4])
def test_multiscale_noise_parity(sess, scales):
    """Multi-scale N0 and N1: the gate pattern bit for bit (exact integer sums
    of the quantised normal against the integer threshold on both sides), T,
    E, I and Y within the bars; odd
    volume sizes exercise the coarse cells' partial edges."""
    wl = synth.ellipsoid_workload(seed=20 + scales, n_envs=2)
    for v in wl.volumes:
        v.noise_scales = scales
    check_all(sess, wl, name=f"S={scales}")
    lab = np.zeros((37, 29, 41), dtype=np.uint8)
    lab[:, :, :] = 1
    lab[20:, :, :] = 3
    vol = Volume(labels=lab, seed=99, noise_scales=scales)
    t = table_with(mu1_1=0.3, mu1_3=-0.2)
    wl2 = single_env(vol, Probe(W=45, H=70, dx=0.7, dy=0.45), axis_pose((20.0, 14.0, 1.0)), t)
    check_all(sess, wl2, name=f"S={scales} odd")


def test_volumetric_probe_parity(sess):
    """Volumetric probe of the surgery task (50 x 37 x 5 at 2 x 2 x 10 mm):
    every elevation plane against the oracle, on the spine phantom and on a
    small volume where outer planes leave the grid."""
    wl = synth.volumetric_workload(seed=2, n_envs=3, n_vols=1)
    g = check_all(sess, wl, name="volumetric")
    assert g[0]["Y"].shape == (5, 50, 37)
    vol = Volume(labels=synth.ellipsoid_volume(5), seed=3)
    wl2 = single_env(vol, Probe(W=30, H=60, n_elev=7, elev=9.0), axis_pose((32.0, 32.0, 2.0)))
    check_all(sess, wl2, name="volumetric small")


def test_gate_extremes_and_energy_scale(sess):
    table = synth.default_tissue_table().copy()
    table[1, 4] = np.inf     # soft tissue always scatters
    table[2, 4] = -np.inf    # fat never
    wl = synth.ellipsoid_workload(seed=11, n_envs=3)
    wl.table = table
    for p in wl.probes:
        p.E0 = 3.5
        p.dr = 45.0
    check_all(sess, wl, name="gate")


def test_many_labels_and_permutation(sess):
    rng = np.random.default_rng(5)
    lab = rng.integers(0, 9, size=(24, 24, 24)).astype(np.uint8)
    t = np.zeros((9, 5), dtype=np.float32)
    t[:, 0] = rng.uniform(0.5, 8.0, 9)
    t[0, 0] = 0.0
    t[:, 1] = rng.uniform(0.0, 1.0, 9)
    t[:, 2] = rng.uniform(0.0, 0.1, 9)
    t[:, 3] = rng.uniform(0.0, 0.05, 9)
    t[:, 4] = rng.uniform(-1, 1, 9)
    vol = Volume(labels=lab, spacing=(0.8, 1.0, 1.2), seed=77)
    pose = synth.pose_from(synth.random_rotation(rng), (10.0, 12.0, 11.0))
    wl = single_env(vol, Probe(W=50, H=90, dx=0.3, dy=0.3), pose, t)
    check_all(sess, wl, name="9 labels")


def test_ct_impedance_parity(sess):
    """Spine phantom with an int16 CT volume (impedance from HU)."""
    wl = synth.spine_ct_workload(seed=3, n_envs=6, dims=(128, 128, 128), W=64, H=128)
    g = check_all(sess, wl, name="ct")
    assert any((x["label"] == 3).any() for x in g)


def test_spine_ct_256_cubed_64_envs_full_size(sess):
    """Full-size CT workload: 256^3 labels + int16 HU, 64 envs, 128 x 256."""
    wl = synth.spine_ct_workload(seed=0)
    assert wl.n_envs == 64 and wl.volumes[0].labels.shape == (256, 256, 256)
    check_all(sess, wl, name="c2")


def test_error_paths(sess):
    from paper_2507_01152_amd import sonosim as sg
    wl = synth.ellipsoid_workload(seed=1, n_envs=1)
    vids = sess.load(wl)
    out, offs = sess.frames(wl)

    def sim(**kw):
        args = dict(vol_ids=vids, probes=wl.probes, poses=wl.poses, out=out, out_offsets=offs)
        args.update(kw)
        sg.sg_simulate(sess.ctx, **args)

    bad_pose = wl.poses.copy()
    bad_pose[0, 3] = np.nan
    with pytest.raises(sg.SonosimError) as e:
        sim(poses=bad_pose)
    assert e.value.status == sg.SG_EINVAL
    far = wl.poses.copy()
    far[0, 3] = 1e9
    with pytest.raises(sg.SonosimError) as e:
        sim(poses=far)
    assert e.value.status == sg.SG_ERANGE
    with pytest.raises(sg.SonosimError) as e:
        sim(probes=[Probe(W=0, H=10)])
    assert e.value.status == sg.SG_EINVAL
    with pytest.raises(sg.SonosimError) as e:
        sim(probes=[Probe(W=64, H=128, psf=0.2)])       # PSF radius > 32 px
    assert e.value.status == sg.SG_EINVAL
    with pytest.raises(sg.SonosimError) as e:
        sim(vol_ids=[1234])
    assert e.value.status == sg.SG_EINVAL
    # a table smaller than the volume's labels
    sg.sg_tissue_table_set(sess.ctx, wl.table[:2])
    with pytest.raises(sg.SonosimError) as e:
        sim()
    assert e.value.status == sg.SG_EINVAL
    sg.sg_tissue_table_set(sess.ctx, wl.table)
    sim()
    torch.cuda.synchronize()


def test_odd_volume_dims_random_labels(sess):
    """A label volume whose sides are not multiples of the 8 x 4 x 4-voxel
    bricks, with a random label per voxel, cut by an oblique plane that also
    leaves it: every pixel's label and voxel index (and the frame) against the
    oracle."""
    rng = np.random.default_rng(11)
    vol = Volume(labels=rng.integers(1, 4, size=(29, 13, 37), dtype=np.uint8), seed=5)
    a, b = 0.6, 0.12
    Ry = np.array([[np.cos(a), 0, np.sin(a)], [0, 1, 0], [-np.sin(a), 0, np.cos(a)]])
    Rx = np.array([[1, 0, 0], [0, np.cos(b), -np.sin(b)], [0, np.sin(b), np.cos(b)]])
    wl = single_env(vol, Probe(W=90, H=100, dx=0.45, dy=0.4), axis_pose((-3.0, 4.0, -2.0), Ry @ Rx))
    g = check_all(sess, wl, name="odd dims")
    assert (g[0]["voxel"] == -1).any() and (g[0]["voxel"] >= 0).any()
    assert len(np.unique(g[0]["label"])) >= 3


def test_registration_copies_the_label_map(sess):
    """The library keeps its own (bricked) copy of a label map: later changes
    to the caller's buffer do not reach the frames, and a released volume is
    refused."""
    from paper_2507_01152_amd import sonosim as sg
    wl = synth.ellipsoid_workload(seed=3, n_envs=1)
    v = wl.volumes[0]
    lab = torch.from_numpy(np.ascontiguousarray(v.labels)).to(sess.device)
    vid = sg.sg_volume_register(sess.ctx, lab, v.spacing, None, v.seed, 1)
    sg.sg_tissue_table_set(sess.ctx, wl.table)
    out, offs = sess.frames(wl)
    ids = np.asarray([vid], dtype=np.int32)
    sg.sg_simulate(sess.ctx, ids, wl.probes, wl.poses, out, offs)
    torch.cuda.synchronize()
    first = out.clone()
    assert (first > 0).any()
    lab.fill_(2)
    out.zero_()
    sg.sg_simulate(sess.ctx, ids, wl.probes, wl.poses, out, offs)
    torch.cuda.synchronize()
    assert torch.equal(out, first)
    sg.sg_volume_release(sess.ctx, vid)
    with pytest.raises(sg.SonosimError) as e:
        sg.sg_simulate(sess.ctx, ids, wl.probes, wl.poses, out, offs)
    assert e.value.status == sg.SG_EINVAL
    with pytest.raises(sg.SonosimError):
        sg.sg_volume_release(sess.ctx, vid)


@pytest.mark.parametrize("scales", [1, 3])
def test_fast_and_general_ray_paths_agree_bit_for_bit(sess, scales):
    """Label volumes without debug planes run the ray kernel's label-only
    instantiation; with debug planes (as in the oracle parity cases) they run
    the general one.  Both must give the same frames bit for bit."""
    import dataclasses
    wl = synth.ellipsoid_workload(seed=5, n_envs=6)
    wl = dataclasses.replace(wl, volumes=[dataclasses.replace(v, noise_scales=scales) for v in wl.volumes])
    vids = sess.load(wl)
    fast, _, _ = sess.simulate(wl, vids, debug=False)
    general, _, dbg = sess.simulate(wl, vids, debug=True)
    torch.cuda.synchronize()
    assert torch.equal(fast, general)
    assert (fast > 0).any()


@pytest.mark.parametrize("dims", [(1, 1, 1), (5, 1, 3), (9, 5, 2)])
def test_volumes_smaller_than_a_brick(sess, dims):
    """Label volumes smaller than (or straddling) one 8 x 4 x 4-voxel brick:
    the padding of the bricked copy must never be read as a voxel.  Labels,
    voxel indices and the frame against the oracle, with the plane crossing
    the whole volume and leaving it."""
    nx, ny, nz = dims
    rng = np.random.default_rng(nx * 100 + ny * 10 + nz)
    vol = Volume(labels=rng.integers(1, 4, size=(nz, ny, nx), dtype=np.uint8), seed=9)
    # scanlines along x, beam along z, through the middle of y; 0.3 mm pixels reach past every side
    pose = axis_pose((-0.9, (ny - 1) / 2.0, -0.8))
    wl = single_env(vol, Probe(W=int(nx / 0.3) + 8, H=int(nz / 0.3) + 8, dx=0.3, dy=0.3), pose)
    g = check_all(sess, wl, name=f"tiny {dims}")
    assert (g[0]["voxel"] >= 0).sum() >= nx * nz and (g[0]["voxel"] == -1).any()


def _many_label_workload(n_labels, scales, seed=31):
    """A 40^3 volume of random labels 0..n_labels-1 in blocks of 3 voxels
    (boundaries along every axis) under a random table, imaged by an oblique
    plane: more than 16 labels leave the label-pair table unused, so the ray
    kernel takes the FP64 impedance path."""
    rng = np.random.default_rng(seed)
    blocks = rng.integers(0, n_labels, size=(14, 14, 14)).astype(np.uint8)
    lab = np.ascontiguousarray(blocks.repeat(3, 0).repeat(3, 1).repeat(3, 2)[:40, :40, :40])
    lab[0, 0, 0] = n_labels - 1
    t = np.zeros((n_labels, 5), dtype=np.float32)
    t[:, 0] = rng.uniform(0.5, 8.0, n_labels)
    t[0, 0] = 0.0
    t[1, 0] = np.inf
    t[:, 1] = rng.uniform(0.0, 0.8, n_labels)
    t[:, 2] = rng.uniform(0.0, 0.1, n_labels)
    t[:, 3] = rng.uniform(0.0, 0.05, n_labels)
    t[:, 4] = rng.uniform(-1, 1, n_labels)
    vol = Volume(labels=lab, spacing=(0.9, 1.0, 1.1), seed=78, noise_scales=scales)
    poses = np.stack([synth.pose_from(synth.random_rotation(rng), (18.0 + i, 20.0, 17.0 - i)) for i in range(3)])
    probes = [Probe(W=70, H=150, dx=0.3, dy=0.25), Probe(W=33, H=64, dx=0.4, dy=0.5),
              Probe(W=129, H=97, dx=0.2, dy=0.3)]
    return Workload([vol], np.zeros(3, dtype=np.int32), probes, poses, t)


@pytest.mark.parametrize("scales", [1, 3])
def test_many_labels_without_debug_planes(sess, scales):
    """20 labels (no label-pair table) launched without debug planes: the
    ray kernel's non-label-only, non-debug instantiation.  Frames against the
    oracle, and bit for bit against the debug instantiation (itself checked
    against the oracle plane by plane)."""
    wl = _many_label_workload(20, scales)
    g = check_all(sess, wl, name=f"20 labels S={scales} fast", debug=False)
    assert any(len(np.unique(np.round(x["Y"], 3))) > 50 for x in g)
    check_all(sess, wl, name=f"20 labels S={scales} debug")
    vids = sess.load(wl)
    fast, _, _ = sess.simulate(wl, vids, debug=False)
    general, _, _ = sess.simulate(wl, vids, debug=True)
    torch.cuda.synchronize()
    assert torch.equal(fast, general)


def test_spine_ct_full_size_without_debug_planes(sess):
    """The full-size CT workload (64 envs, 256^3 labels + int16 HU, 128 x 256)
    without debug planes: the CT instantiation the batched CT physics and the
    CT surrogate's targets run on.  Every env's frame against the oracle, and
    bit for bit against the debug instantiation."""
    wl = synth.spine_ct_workload(seed=0)
    check_all(sess, wl, name="c2 fast", debug=False)
    vids = sess.load(wl)
    fast, _, _ = sess.simulate(wl, vids, debug=False)
    general, _, _ = sess.simulate(wl, vids, debug=True)
    torch.cuda.synchronize()
    assert torch.equal(fast, general) and (fast > 0).any()
