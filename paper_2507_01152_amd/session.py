"""Device-side bookkeeping around the C ABI: uploads volumes to device
tensors, registers them, allocates packed output frames.  Marshalling only."""
from __future__ import annotations

import numpy as np
import torch

from . import sonosim as sg


class Session:
    def __init__(self, device: int = 0, stream=None):
        self.device = torch.device("cuda", device)
        self.ctx = sg.sg_create(device, stream)
        self._keep = []

    def close(self):
        if self.ctx is not None:
            sg.sg_destroy(self.ctx)
            self.ctx = None
        self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def register(self, volume) -> int:
        lab = torch.from_numpy(np.ascontiguousarray(volume.labels)).to(self.device)
        ct = None
        if volume.ct is not None:
            ct = torch.from_numpy(np.ascontiguousarray(volume.ct)).to(self.device)
        self._keep.append((lab, ct))
        return sg.sg_volume_register(self.ctx, lab, volume.spacing, ct, volume.seed,
                                     getattr(volume, "noise_scales", 1))

    def load(self, workload):
        """Register the workload's volumes and tissue table; returns env vol ids."""
        ids = [self.register(v) for v in workload.volumes]
        sg.sg_tissue_table_set(self.ctx, workload.table)
        return np.asarray([ids[i] for i in workload.vol_ids], dtype=np.int32)

    def frames(self, workload):
        offs, total = workload.out_offsets()
        return torch.empty(total, dtype=torch.float32, device=self.device), offs

    def debug_planes(self, total: int):
        d = self.device
        return {
            "label": torch.empty(total, dtype=torch.uint8, device=d),
            "voxel": torch.empty(total, dtype=torch.int32, device=d),
            "philox": torch.empty(4 * total, dtype=torch.int32, device=d),
            "energy": torch.empty(total, dtype=torch.float32, device=d),
            "intensity": torch.empty(total, dtype=torch.float32, device=d),
            "scatter": torch.empty(total, dtype=torch.float32, device=d),
        }

    def simulate(self, workload, vol_ids, debug: bool = False):
        out, offs = self.frames(workload)
        dbg = self.debug_planes(out.numel()) if debug else None
        sg.sg_simulate(self.ctx, vol_ids, workload.probes, workload.poses, out, offs, dbg)
        return out, offs, dbg


def split_frames(flat: np.ndarray, workload, per_pixel: int = 1):
    """Unpack a packed buffer into per-env [H][W] (or [H][W][k]) arrays;
    volumetric probes give [E][H][W] (or [E][H][W][k])."""
    offs, _ = workload.out_offsets()
    res = []
    for o, p in zip(offs, workload.probes):
        E = max(1, int(getattr(p, "n_elev", 1)))
        n = p.W * p.H * E
        a = flat[per_pixel * o: per_pixel * (o + n)]
        shape = (p.H, p.W) if per_pixel == 1 else (p.H, p.W, per_pixel)
        res.append(a.reshape(((E,) if E > 1 else ()) + shape))
    return res
