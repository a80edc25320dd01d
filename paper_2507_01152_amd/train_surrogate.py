"""Train the surrogate on pairs rendered by the physics path.

Workload: seeded 64^3 ellipsoid label phantoms (1 mm voxels), imaged at
128 scanlines x 256 depth samples with 0.25 mm pixels from random poses;
every step draws a fresh batch of (phantom, pose) pairs and the library
renders the targets and encodes the inputs on the GPU.  Held-out phantoms
measure the PSNR of the network against the physics frames (through the
audited inference path).

The CT-conditioned surrogate (train_ct) learns from 256^3 spine phantoms
with CT, 128 x 256 frames at 0.5 mm, histogram-matched CT input and the
adversarial term.

    python -m paper_2507_01152_amd.train_surrogate --steps 3000 --batch 64 --ckpt surr.bin
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FRAME_W, FRAME_H, PIXEL_MM = 128, 256, 0.25


class PairSource:
    """Phantoms registered on the device and a seeded pose generator."""

    def __init__(self, sess, n_volumes: int, seed0: int):
        import synth
        from . import sonosim as sg
        self.synth = synth
        vols = [synth.Volume(labels=synth.ellipsoid_volume(seed0 + i), seed=0x5EED0000 + seed0 + i)
                for i in range(n_volumes)]
        self.ids = np.array([sess.register(v) for v in vols], dtype=np.int32)
        sg.sg_tissue_table_set(sess.ctx, synth.default_tissue_table())
        self.probe = synth.Probe(W=FRAME_W, H=FRAME_H, dx=PIXEL_MM, dy=PIXEL_MM)

    def batch(self, n: int, rng: np.random.Generator):
        s = self.synth
        vids = self.ids[rng.integers(0, len(self.ids), n)]
        poses = np.stack([s.pose_from(s.random_rotation(rng), rng.uniform(16, 48, 3)) for _ in range(n)])
        return vids, [self.probe] * n, poses


CT_FRAME_W, CT_FRAME_H, CT_PIXEL_MM, CT_DIMS = 128, 256, 0.5, (256, 256, 256)


class CtPairSource:
    """Spine phantoms with CT (256^3 labels + int16 HU, 1 mm voxels) on the
    device and probe poses on the back (the CT workload's pose sampler)."""

    def __init__(self, sess, n_volumes: int, seed0: int):
        import synth
        from . import sonosim as sg
        self.synth = synth
        self.geoms, ids = [], []
        for i in range(n_volumes):
            lab, geom = synth.spine_volume(CT_DIMS, seed0 + i)
            vol = synth.Volume(labels=lab, ct=synth.ct_from_labels(lab, seed0 + i), seed=0xC7000000 + seed0 + i)
            ids.append(sess.register(vol))
            self.geoms.append(geom)
        self.ids = np.array(ids, dtype=np.int32)
        sg.sg_tissue_table_set(sess.ctx, synth.default_tissue_table())
        self.probe = synth.Probe(W=CT_FRAME_W, H=CT_FRAME_H, dx=CT_PIXEL_MM, dy=CT_PIXEL_MM)

    def batch(self, n: int, rng: np.random.Generator):
        k = rng.integers(0, len(self.ids), n)
        poses = np.stack([self.synth.spine_pose(self.geoms[i], CT_DIMS[1], rng) for i in k])
        return self.ids[k], [self.probe] * n, poses


def train_ct(steps: int, batch: int, lr: float, adv_weight: float = 0.01, seed: int = 0, n_train_vols: int = 16,
             n_ref_frames: int = 64, log=print):
    """CT-conditioned surrogate with the adversarial term: the histogram
    reference is pooled over n_ref_frames training frames, then every step
    draws a fresh batch of (phantom, pose) pairs.  Returns (session,
    surrogate id, training source, per-step wall seconds, last losses)."""
    from . import sonosim as sg
    from .session import Session
    sess = Session(0)
    src = CtPairSource(sess, n_train_vols, seed0=7000)
    sid = sg.sg_surr_create_ct(sess.ctx, CT_FRAME_H, CT_FRAME_W, seed=seed, adv_weight=adv_weight)
    rng = np.random.default_rng(seed + 11)
    sg.sg_surr_set_ct_reference(sess.ctx, sid, *src.batch(n_ref_frames, rng))
    t0 = time.time()
    last = None
    first = sg.sg_surr_step_count(sess.ctx, sid)
    for step in range(1, steps + 1):
        cur = lr if step < 0.7 * steps else lr * 0.1
        # enqueued without a loss readback; the losses are read from the device's log when reported
        sg.sg_surr_train_step_async(sess.ctx, sid, *src.batch(batch, rng), cur)
        if step == steps or step % 200 == 0:
            l1, ld, la = (float(v) for v in sg.sg_surr_loss_history(sess.ctx, sid, first + step, 1)[0])
            last = {"step": step, "l1": round(l1, 5), "loss_d": round(ld, 4), "loss_adv": round(la, 4),
                    "wall_s": round(time.time() - t0, 1)}
            log(json.dumps(last))
    return sess, sid, src, (time.time() - t0) / max(1, steps), last


def evaluate(sess, sid, src: PairSource, n: int = 64, seed: int = 123):
    """Mean and pooled PSNR (dB) of the network against physics on n envs."""
    import torch
    from . import sonosim as sg
    rng = np.random.default_rng(seed)
    vids, probes, poses = src.batch(n, rng)
    out = torch.empty(n * FRAME_W * FRAME_H, dtype=torch.float32, device=sess.device)
    psnr, _ = sg.sg_surr_infer(sess.ctx, sid, vids, probes, poses, out, list(range(n)), -np.inf, 1.0)
    mse = 10.0 ** (-np.asarray(psnr, dtype=np.float64) / 10.0)
    return float(np.mean(psnr)), float(-10.0 * np.log10(mse.mean()))


def train(steps: int, batch: int, lr: float, seed: int = 0, eval_every: int = 500, ckpt: str | None = None,
          resume: str | None = None, n_train_vols: int = 256, log=print):
    from . import sonosim as sg
    from .session import Session
    sess = Session(0)
    train_src = PairSource(sess, n_train_vols, seed0=0)
    eval_src = PairSource(sess, 32, seed0=100000)
    sid = sg.sg_surr_create(sess.ctx, FRAME_H, FRAME_W, seed=seed)
    if resume:
        sg.sg_surr_load(sess.ctx, sid, resume)
    rng = np.random.default_rng(seed + 1)
    history = []
    t0 = time.time()
    first = sg.sg_surr_step_count(sess.ctx, sid)
    for step in range(1, steps + 1):
        # constant rate, then a tenfold decay over the last 30 %
        cur = lr if step < 0.7 * steps else lr * 0.1
        vids, probes, poses = train_src.batch(batch, rng)
        # enqueued without a loss readback (the host draws the next batch meanwhile)
        sg.sg_surr_train_step_async(sess.ctx, sid, vids, probes, poses, cur)
        if step % eval_every == 0 or step == steps:
            loss = float(sg.sg_surr_loss_history(sess.ctx, sid, first + step, 1)[0, 0])
            mean_db, pooled_db = evaluate(sess, sid, eval_src)
            rec = {"step": step, "pairs": step * batch, "loss": round(loss, 5), "psnr_mean_db": round(mean_db, 2),
                   "psnr_pooled_db": round(pooled_db, 2), "wall_s": round(time.time() - t0, 1)}
            history.append(rec)
            log(json.dumps(rec))
    if ckpt:
        sg.sg_surr_save(sess.ctx, sid, ckpt)
    return sess, sid, train_src, eval_src, history


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eval-every", type=int, default=500)
    ap.add_argument("--ckpt", default=None)
    ap.add_argument("--resume", default=None)
    a = ap.parse_args()
    sess, *_ = train(a.steps, a.batch, a.lr, a.seed, a.eval_every, a.ckpt, a.resume,
                     log=lambda s: print(s, flush=True))
    sess.close()


if __name__ == "__main__":
    main()
