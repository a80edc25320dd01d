"""FP64 CPU oracle of the model-based ultrasound simulator (test infrastructure).

Only the tests, the package's smoke check and the benchmark's CPU-baseline leg
may import this package.  It wraps the plain C library built from
``sonosim_oracle.c`` (gcc, FP64, no FMA contraction) with ctypes and shares no
code with the GPU path.  See the C file's header for what each step computes
and which passage of the paper (App. B.2) it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sonosim_oracle.c")
_LIB = os.path.join(_HERE, "_build", "libsonooracle.so")


def build(force: bool = True, sanitize: bool = False, out: str | None = None) -> str:
    """Compile the oracle with gcc (FP64, -ffp-contract=off, OpenMP).  sanitize: an
    AddressSanitizer + UndefinedBehaviorSanitizer build (any finding aborts) into `out`,
    for the sanitizer test; a process loads it through SONO_ORACLE_LIB."""
    path = out or _LIB
    if force or not os.path.exists(path):
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        extra = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                 "-fno-sanitize-recover=undefined"] if sanitize else []
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off", "-fPIC"] + extra +
            ["-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, path)
    return path


class _Volume(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("sx", C.c_double), ("sy", C.c_double), ("sz", C.c_double),
                ("labels", C.c_void_p), ("ct", C.c_void_p), ("seed", C.c_uint64),
                ("scales", C.c_int32), ("q_lut", C.c_void_p)]


class _Tissue(C.Structure):
    _fields_ = [("Z", C.c_float), ("alpha", C.c_float), ("mu0", C.c_float),
                ("sigma0", C.c_float), ("mu1", C.c_float)]


class _Probe(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("dx", C.c_double), ("dy", C.c_double),
                ("f", C.c_double), ("E0", C.c_double), ("psf", C.c_double), ("dr", C.c_double),
                ("elev", C.c_double)]


_PLANES = [("q", np.int64, 3), ("label", np.uint8, 1), ("voxel", np.int64, 1),
           ("philox", np.uint32, 4), ("Z", np.float64, 1), ("G", np.uint8, 1),
           ("r", np.float64, 1), ("t", np.float64, 1), ("E", np.float64, 1),
           ("cos_theta", np.float64, 1), ("T", np.float64, 1), ("Rp", np.float64, 1),
           ("I", np.float64, 1), ("A", np.float64, 1), ("Y", np.float64, 1)]


class _Planes(C.Structure):
    _fields_ = [(name, C.c_void_p) for name, _, _ in _PLANES]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("SONO_ORACLE_LIB") or _LIB
        if path == _LIB and not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(path)
        L.or_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_philox4x64_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_philox4x32_rounds.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
        L.or_philox4x64_rounds.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
        L.or_geometry.argtypes = [C.POINTER(_Volume), C.POINTER(_Probe), C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_gate_threshold.argtypes = [C.c_float]
        L.or_gate_threshold.restype = C.c_uint64
        L.or_psf_kernel.argtypes = [C.c_double, C.c_void_p, C.c_int32]
        L.or_psf_kernel.restype = C.c_int32
        L.or_simulate_env.argtypes = [C.POINTER(_Volume), C.c_void_p, C.c_int32, C.POINTER(_Probe),
                                      C.c_void_p, C.POINTER(_Planes)]
        L.or_simulate_env.restype = C.c_int
        L.or_multiscale_threshold.argtypes = [C.c_int32, C.c_float]
        L.or_multiscale_threshold.restype = C.c_int64
        L.or_scatter_voxel.argtypes = [C.POINTER(_Volume), C.c_float, C.c_int64, C.c_int64, C.c_int64,
                                       C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_void_p]
        L.or_scatter_voxel.restype = C.c_int
        L.or_scatter_grid.argtypes = [C.POINTER(_Volume), C.c_float, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_recon_points.argtypes = [C.POINTER(_Volume), C.c_void_p, C.POINTER(_Probe), C.c_void_p, C.c_int32,
                                      C.c_int32, C.c_int32, C.c_uint64, C.c_double, C.c_void_p]
        L.or_recon_points.restype = C.c_int64
        L.or_recon_observe.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.or_simulate_batch.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                        C.POINTER(C.c_int32)]
        L.or_simulate_batch.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


_Q_LUT = None


def quantised_normal_table() -> np.ndarray:
    """Q[k] = rint(Phi^-1((k + 1/2) / 4096) * 2^20) (int32), k < 4096: the
    quantised standard normal of the multi-scale gate in units of 2^-20
    (scipy's ndtri in FP64, scaled exactly, rounded half to even once)."""
    global _Q_LUT
    if _Q_LUT is None:
        from scipy.special import ndtri
        q = np.rint(ndtri((np.arange(4096) + 0.5) / 4096.0) * 1048576.0)
        _Q_LUT = np.ascontiguousarray(q.astype(np.int32))
    return _Q_LUT


def multiscale_threshold(scales: int, mu1: float) -> int:
    """Integer threshold of the multi-scale gate: floor(sqrt(S) * mu1 * 2^20)
    in FP64, clamped to the int32 range (mu1 is taken as an FP32 value)."""
    return int(lib().or_multiscale_threshold(int(scales), float(mu1)))


def _volume_struct(vol):
    labels = np.ascontiguousarray(vol.labels, dtype=np.uint8)
    ct = None if vol.ct is None else np.ascontiguousarray(vol.ct, dtype=np.int16)
    nz, ny, nx = labels.shape
    sx, sy, sz = vol.spacing
    q = quantised_normal_table()
    s = _Volume(nx, ny, nz, sx, sy, sz, labels.ctypes.data,
                None if ct is None else ct.ctypes.data, int(vol.seed) & ((1 << 64) - 1),
                int(getattr(vol, "noise_scales", 1)), q.ctypes.data)
    return s, (labels, ct, q)


def _table(table):
    t = np.ascontiguousarray(np.asarray(table, dtype=np.float32).reshape(-1, 5))
    return t, t.shape[0]


def n_planes(p) -> int:
    """Image planes of a probe (volumetric probes have n_elev > 1)."""
    return max(1, int(getattr(p, "n_elev", 1)))


def plane_elevation(p, j: int) -> float:
    """Elevation b of plane j, mm: (j - (E - 1) / 2) * spacing, centred."""
    if n_planes(p) == 1:
        return 0.0
    return (float(j) - 0.5 * float(p.n_elev - 1)) * float(p.elev)


def _probe_struct(p, plane: int = 0):
    return _Probe(int(p.W), int(p.H), float(p.dx), float(p.dy), float(p.f), float(p.E0),
                  float(p.psf), float(p.dr), plane_elevation(p, plane))


# ---------------------------------------------------------------------------

def scatter_voxel(vol, mu1: float, ix: int, iy: int, iz: int):
    """Scattering draw of one voxel: (N0 (FP64), N1 (integer sum of the
    quantised normals, units of 2^-20; 0 with one scale), gate (bool), scale-0
    Philox words)."""
    vs, keep = _volume_struct(vol)
    n0, n1 = C.c_double(), C.c_int64()
    w = np.zeros(4, dtype=np.uint32)
    g = lib().or_scatter_voxel(C.byref(vs), float(mu1), int(ix), int(iy), int(iz), C.byref(n0), C.byref(n1),
                               w.ctypes.data)
    return float(n0.value), int(n1.value), bool(g), w


def scatter_grid(vol, mu1: float):
    """(N0, N1, gate) of every voxel of vol, each [nz][ny][nx]; N1 is the
    integer sum of the quantised normals (units of 2^-20)."""
    vs, keep = _volume_struct(vol)
    shape = np.asarray(vol.labels).shape
    n0 = np.zeros(shape, dtype=np.float64)
    n1 = np.zeros(shape, dtype=np.int64)
    g = np.zeros(shape, dtype=np.uint8)
    lib().or_scatter_grid(C.byref(vs), float(mu1), n0.ctypes.data, n1.ctypes.data, g.ctypes.data)
    return n0, n1, g.astype(bool)


def philox4x32(ctr, key, rounds: int = 10) -> np.ndarray:
    """Philox4x32-R of one counter (4 x u32) under one key (2 x u32)."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    o = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_rounds(c.ctypes.data, k.ctypes.data, int(rounds), o.ctypes.data)
    return o


def philox4x64(ctr, key, rounds: int = 10) -> np.ndarray:
    """Philox4x64-R (same round structure as the 32-bit generator)."""
    c = np.asarray(ctr, dtype=np.uint64).copy()
    k = np.asarray(key, dtype=np.uint64).copy()
    o = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64_rounds(c.ctypes.data, k.ctypes.data, int(rounds), o.ctypes.data)
    return o


def geometry(vol, probe, pose):
    """O1: Q16 origin P0 and steps DX, DY (int64, voxel units * 2^16)."""
    vs, keep = _volume_struct(vol)
    ps = _probe_struct(probe)
    pose = np.ascontiguousarray(pose, dtype=np.float64)
    P0, DX, DY = (np.zeros(3, dtype=np.int64) for _ in range(3))
    lib().or_geometry(C.byref(vs), C.byref(ps), pose.ctypes.data, P0.ctypes.data, DX.ctypes.data,
                      DY.ctypes.data)
    return P0, DX, DY


def gate_threshold(mu1: float) -> int:
    return int(lib().or_gate_threshold(C.c_float(mu1)))


def psf_kernel(sigma: float) -> np.ndarray:
    K = np.zeros(4096, dtype=np.float64)
    r = lib().or_psf_kernel(float(sigma), K.ctypes.data, 4096)
    if r < 0:
        raise ValueError("PSF radius too large")
    return K[: 2 * r + 1].copy()


def simulate_env(vol, table, probe, pose, planes=("label", "voxel", "philox", "E", "T", "Rp",
                                                  "I", "A", "Y")) -> dict:
    """Simulate one environment; returns the requested per-pixel planes
    shaped [H][W] (philox [H][W][4], q [H][W][3]); a volumetric probe's
    planes are stacked in front: [E][H][W]."""
    if n_planes(probe) > 1:
        per = [_simulate_plane(vol, table, probe, pose, planes, j) for j in range(n_planes(probe))]
        return {k: np.stack([d[k] for d in per]) for k in per[0]}
    return _simulate_plane(vol, table, probe, pose, planes, 0)


def _simulate_plane(vol, table, probe, pose, planes, j):
    vs, keep = _volume_struct(vol)
    t, n_labels = _table(table)
    ps = _probe_struct(probe, j)
    pose = np.ascontiguousarray(pose, dtype=np.float64)
    out, pl = {}, _Planes()
    want = set(planes)
    for name, dt, k in _PLANES:
        if name in want:
            shape = (probe.H, probe.W) if k == 1 else (probe.H, probe.W, k)
            out[name] = np.zeros(shape, dtype=dt)
            setattr(pl, name, out[name].ctypes.data)
    rc = lib().or_simulate_env(C.byref(vs), t.ctypes.data, n_labels, C.byref(ps), pose.ctypes.data,
                               C.byref(pl))
    if rc != 0:
        raise ValueError("oracle rejected the inputs (label outside the table or bad size)")
    return out


def simulate_batch(workload, env_ids=None, n_threads: int = 0):
    """Display frames Y (float64) of the listed envs, OpenMP over envs.
    Returns (list of [H][W] arrays, threads used)."""
    if env_ids is None:
        env_ids = list(range(workload.n_envs))
    vol_structs, keep = [], []
    for v in workload.volumes:
        s, k = _volume_struct(v)
        vol_structs.append(s)
        keep.append(k)
    vols = (_Volume * len(vol_structs))(*vol_structs)
    t, n_labels = _table(workload.table)
    # one oracle env per image plane
    pl = [(e, j) for e in env_ids for j in range(n_planes(workload.probes[e]))]
    probes = (_Probe * len(pl))(*[_probe_struct(workload.probes[e], j) for e, j in pl])
    vol_ids = np.ascontiguousarray([workload.vol_ids[e] for e, _ in pl], dtype=np.int32)
    poses = np.ascontiguousarray(workload.poses[[e for e, _ in pl]], dtype=np.float64)
    sizes = np.array([workload.probes[e].W * workload.probes[e].H for e, _ in pl], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    Y = np.zeros(int(sizes.sum()), dtype=np.float64)
    used = C.c_int32(0)
    rc = lib().or_simulate_batch(len(pl), C.cast(vols, C.c_void_p), vol_ids.ctypes.data,
                                 t.ctypes.data, n_labels, C.cast(probes, C.c_void_p), poses.ctypes.data,
                                 Y.ctypes.data, offs.ctypes.data, int(n_threads), C.byref(used))
    if rc != 0:
        raise ValueError("oracle rejected the inputs")
    frames, k = [], 0
    for e in env_ids:
        p = workload.probes[e]
        E = n_planes(p)
        f = Y[offs[k]:offs[k] + E * p.W * p.H].reshape(E, p.H, p.W)
        frames.append(f if E > 1 else f[0])
        k += E
    return frames, int(used.value)


# ---------------------------------------------------------------------------
# reconstruction observation (bone-surface task)

def recon_points(vol, probe, pose, env: int, step: int, seed: int, p_drop: float = 0.2, bone_labels=(3,)):
    """Kept bone-surface points of one frame (all planes), float64 [n, 3] in volume mm."""
    vs, keep = _volume_struct(vol)
    bone = np.zeros(256, dtype=np.uint8)
    bone[list(bone_labels)] = 1
    pose = np.ascontiguousarray(pose, dtype=np.float64)
    out = []
    for j in range(n_planes(probe)):
        ps = _probe_struct(probe, j)
        buf = np.zeros((probe.W, 3), dtype=np.float64)
        n = lib().or_recon_points(C.byref(vs), bone.ctypes.data, C.byref(ps), pose.ctypes.data, j, int(env),
                                  int(step), int(seed) & ((1 << 64) - 1), float(p_drop), buf.ctypes.data)
        out.append(buf[:n])
    return np.concatenate(out) if out else np.zeros((0, 3))


def recon_observe(points, pose) -> np.ndarray:
    """40^3 occupancy grid (depth, lateral, elevation) of points at a pose."""
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    pose = np.ascontiguousarray(pose, dtype=np.float64)
    grid = np.zeros((40, 40, 40), dtype=np.uint8)
    lib().or_recon_observe(pts.ctypes.data, pts.shape[0], pose.ctypes.data, grid.ctypes.data)
    return grid
