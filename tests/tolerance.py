"""Parity bars between the HIP path (FP32) and the FP64 oracle.

Integer work (nearest label, voxel index, Philox words) must match bit for
bit.  Floating-point quantities must agree within 1e-4 relative:
  E:  |dE| <= 1e-4 * E + 1e-30 * E0
  I:  |dI| <= 1e-4 * A + 1e-30 * E0, A = K(x)R' + E * K(x)|T| (the magnitude
      sum; plain relative error is ill-posed where signed speckle cancels)
  Y:  |dY| <= 1e-4 + (20 / (DR ln 10)) * (1e-4 * A + 1e-30 * E0) / max(I, E0 * 10^(-DR/20))
The 1e-30 * E0 floor covers energies below FP32's normal range, which the
display maps to 0 anyway.
"""
import numpy as np

REL = 1e-4
FLOOR = 1e-30


def check_env(gpu: dict, ora: dict, probe, name: str = ""):
    E0, DR = probe.E0, probe.dr
    if "label" in gpu:
        assert np.array_equal(gpu["label"], ora["label"]), f"{name}: label mismatch"
    if "voxel" in gpu:
        assert np.array_equal(gpu["voxel"].astype(np.int64), ora["voxel"]), f"{name}: voxel mismatch"
    if "philox" in gpu:
        assert np.array_equal(gpu["philox"].view(np.uint32), ora["philox"]), f"{name}: philox mismatch"
    if "energy" in gpu:
        dE = np.abs(gpu["energy"].astype(np.float64) - ora["E"])
        bad = dE > REL * ora["E"] + FLOOR * E0
        assert not bad.any(), f"{name}: E off at {np.argwhere(bad)[:5].tolist()} max rel {(dE / np.maximum(ora['E'], 1e-300)).max():.3g}"
    if "scatter" in gpu and "T" in ora:
        # the density gate is decided identically (integer test, or the FP32
        # sum of quantised normals); the amplitude within FP32 + 1e-5 relative
        Tg = gpu["scatter"].astype(np.float64)
        assert np.array_equal(Tg != 0, ora["T"] != 0), f"{name}: scatter gate mismatch"
        dT = np.abs(Tg - ora["T"])
        bad = dT > 1e-5 * (np.abs(ora["T"]) + 1e-3)
        assert not bad.any(), f"{name}: T off at {np.argwhere(bad)[:5].tolist()}"
    A = ora["A"]
    tolI = REL * A + FLOOR * E0
    if "intensity" in gpu:
        dI = np.abs(gpu["intensity"].astype(np.float64) - ora["I"])
        bad = dI > tolI
        assert not bad.any(), f"{name}: I off at {np.argwhere(bad)[:5].tolist()} worst {(dI / tolI).max():.3g}x tol"
    if "Y" in gpu:
        floor = E0 * 10.0 ** (-DR / 20.0)
        tolY = REL + (20.0 / (DR * np.log(10.0))) * tolI / np.maximum(ora["I"], floor)
        dY = np.abs(gpu["Y"].astype(np.float64) - ora["Y"])
        bad = dY > tolY
        assert not bad.any(), f"{name}: Y off at {np.argwhere(bad)[:5].tolist()} worst {(dY / tolY).max():.3g}x tol"
