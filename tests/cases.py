"""Small hand-built inputs for pins and parity cases (no simulation arithmetic).

Shared by the oracle pin tests and the GPU parity tests so that both sides see
identical inputs.
"""
from __future__ import annotations

import numpy as np

import synth
from synth import Probe, Volume, Workload, pose_from


def axis_pose(t, R=None):
    """Probe x -> volume x, probe z (beam) -> volume z unless R is given."""
    return pose_from(np.eye(3) if R is None else np.asarray(R, dtype=np.float64), t)


def layered_volume(nx, ny, nz, layers, seed=1):
    """Label volume whose label depends only on z: layers = [(z_start, label), ...]."""
    lab = np.zeros((nz, ny, nx), dtype=np.uint8)
    for z0, l in layers:
        lab[z0:] = l
    return Volume(labels=lab, seed=seed)


def table_with(**over):
    """Default tissue table with entries replaced: keyword '<column>_<label>',
    e.g. Z_3=inf sets the impedance of label 3."""
    t = synth.default_tissue_table().copy()
    cols = {"Z": 0, "alpha": 1, "mu0": 2, "sigma0": 3, "mu1": 4}
    for k, v in over.items():
        name, lab = k.rsplit("_", 1)
        t[int(lab), cols[name]] = v
    return t


def single_env(vol, probe, pose, table=None):
    return Workload([vol], np.zeros(1, dtype=np.int32), [probe], np.asarray(pose)[None, :],
                    synth.default_tissue_table() if table is None else table)
