"""The entry point without allocation (sg_simulate_noalloc) against
sg_simulate through the C ABI (GPU): identical frames on two calls in a row,
the second smaller, and refusals beyond its limits."""
import numpy as np
import pytest

import synth
from synth import Probe, Workload

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


def _both(sess, wl):
    from paper_2507_01152_amd import sonosim as sg
    vids = sess.load(wl)
    ref, offs = sess.frames(wl)
    sg.sg_simulate(sess.ctx, vids, wl.probes, wl.poses, ref, offs)
    out = torch.full_like(ref, -1.0)
    sg.sg_simulate_noalloc(sess.ctx, vids, wl.probes, wl.poses, out, offs)
    torch.cuda.synchronize()
    return ref, out


def test_noalloc_matches_simulate_on_two_calls(sess):
    """A label batch with a volumetric probe and uneven frames, then a smaller
    CT batch (the other ray instantiation): the second call reuses the array
    the first one left behind and must still give sg_simulate's frames."""
    a = synth.ellipsoid_workload(seed=13, n_envs=5)
    v = synth.volumetric_workload(seed=2, n_envs=2, n_vols=1)
    probes = list(a.probes) + list(v.probes) + [Probe(W=200, H=333, dx=0.2, dy=0.15)]
    wl1 = Workload(a.volumes + v.volumes, np.array([0, 1, 2, 3, 4, 5, 5, 0], dtype=np.int32), probes,
                   np.concatenate([a.poses, v.poses, a.poses[:1]]), a.table)
    ref, out = _both(sess, wl1)
    assert torch.equal(out, ref) and (ref > 0).any()
    wl2 = synth.spine_ct_workload(seed=5, n_envs=3, dims=(96, 96, 96), W=48, H=90)
    ref2, out2 = _both(sess, wl2)
    assert ref2.numel() < ref.numel()
    assert torch.equal(out2, ref2) and (ref2 > 0).any()


def test_noalloc_refuses_calls_beyond_its_scratch(sess):
    from paper_2507_01152_amd import sonosim as sg
    wl = synth.ellipsoid_workload(seed=14, n_envs=6, W=1024, H=1024, dx=0.06, dy=0.06)
    vids = sess.load(wl)
    out, offs = sess.frames(wl)
    with pytest.raises(sg.SonosimError) as e:     # 6.3 M field pixels: 75 MB of fields
        sg.sg_simulate_noalloc(sess.ctx, vids, wl.probes, wl.poses, out, offs)
    assert e.value.status == sg.SG_ERANGE
    many = synth.ellipsoid_workload(seed=15, n_envs=257, W=8, H=8)
    vids = sess.load(many)
    out, offs = sess.frames(many)
    with pytest.raises(sg.SonosimError) as e:
        sg.sg_simulate_noalloc(sess.ctx, vids, many.probes, many.poses, out, offs)
    assert e.value.status == sg.SG_ERANGE
    # a call within the limits still works after the refusals
    small = synth.ellipsoid_workload(seed=16, n_envs=2, W=30, H=40)
    ref, out = _both(sess, small)
    assert torch.equal(out, ref)
