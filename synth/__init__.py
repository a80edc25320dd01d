"""Seeded synthetic inputs for the ultrasound simulator.

This module is shared by the HIP path's tests/benchmark and by the FP64 oracle.
It holds *no* arithmetic of the simulation method itself: it only paints label
volumes, draws CT numbers, draws probe poses and image sizes, and provides the
tissue parameter table.  Everything the simulator computes from these inputs
(plane geometry, sampling, reflection, energy, speckle, PSF, display) lives in
the two independent implementations.

The paper simulates on CT volumes and label maps of TotalSegmentator patients
(Sec. 4, "Assets"; App. B.1) which are not available here.  The generators
below stand in for them with the same structure: a uint8 label map
(0 air, 1 soft tissue, 2 fat, 3 bone), an optional int16 CT volume whose HU
values are drawn per label, a spine-like chain of bone ellipsoids under the
back skin, and probe poses on the back of the body.

Volumes are numpy arrays indexed [z][y][x] (x fastest in memory), with 1 mm
isotropic voxel spacing.  A pose is 12 float64 values, a row-major 3x4 [R|t]
that maps probe-frame millimetres to volume millimetres (origin at the centre
of voxel (0,0,0)); probe x is the lateral (scanline) axis, probe z the beam.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# label ids
AIR, SOFT, FAT, BONE = 0, 1, 2, 3

# HU means per label used to draw the CT-like volume (sd 30 HU).
HU_MEAN = (-1000.0, 40.0, -100.0, 700.0)
HU_SD = 30.0


def default_tissue_table() -> np.ndarray:
    """Per-label parameters (Z [MRayl], alpha [Np/cm/MHz], mu0, sigma0, mu1).

    The paper takes attenuation and scattering parameters from a commercial
    tool's presets (App. B.2) without printing them; these values are this
    project's own choice (typical soft-tissue/fat/bone impedances and
    attenuations).  Air has Z = 0 (pressure-release) and mu1 = -inf (never
    scatters).  Returned as float32 array of shape (4, 5).
    """
    return np.array(
        [
            [0.0, 0.0, 0.0, 0.0, -np.inf],   # air
            [1.63, 0.062, 0.05, 0.02, 0.0],  # soft tissue
            [1.38, 0.055, 0.03, 0.015, -0.5],  # fat
            [7.8, 2.3, 0.08, 0.03, 0.5],     # bone
        ],
        dtype=np.float32,
    )


@dataclass
class Probe:
    """Linear probe / image geometry of one environment."""
    W: int          # scanlines (image columns)
    H: int          # depth samples (image rows)
    dx: float = 0.5  # lateral pixel pitch, mm
    dy: float = 0.5  # axial pixel pitch, mm
    f: float = 5.0   # frequency, MHz
    E0: float = 1.0  # initial energy
    psf: float = 0.01  # PSF std as a fraction of the image size
    dr: float = 60.0   # display dynamic range, dB
    n_elev: int = 1    # planes of a volumetric probe
    elev: float = 0.0  # plane spacing along the elevation, mm

    @property
    def planes(self) -> int:
        return max(1, int(self.n_elev))

    def astuple(self):
        return (self.W, self.H, self.dx, self.dy, self.f, self.E0, self.psf, self.dr)


@dataclass
class Volume:
    labels: np.ndarray            # uint8 [nz][ny][nx]
    ct: np.ndarray | None = None  # int16 [nz][ny][nx] or None
    spacing: tuple = (1.0, 1.0, 1.0)  # mm along (x, y, z)
    seed: int = 0                 # noise-field key
    noise_scales: int = 1         # scales of the noise field (1: one sample per voxel)

    @property
    def dims(self):
        nz, ny, nx = self.labels.shape
        return nx, ny, nz


@dataclass
class Workload:
    volumes: list
    vol_ids: np.ndarray           # int32 [n_envs]
    probes: list                  # Probe per env
    poses: np.ndarray             # float64 [n_envs, 12]
    table: np.ndarray = field(default_factory=default_tissue_table)

    @property
    def n_envs(self):
        return len(self.probes)

    def out_offsets(self):
        sizes = np.array([p.W * p.H * p.planes for p in self.probes], dtype=np.int64)
        offs = np.zeros(len(sizes), dtype=np.int64)
        if len(sizes) > 1:
            offs[1:] = np.cumsum(sizes)[:-1]
        return offs, int(sizes.sum())


# ---------------------------------------------------------------------------
# rotations

def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly distributed rotation (normalised Gaussian quaternion)."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array(
        [
            [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
            [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
            [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
        ]
    )


def _rot_axis(axis: int, ang: float) -> np.ndarray:
    c, s = math.cos(ang), math.sin(ang)
    if axis == 0:
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    if axis == 1:
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def pose_from(R: np.ndarray, t) -> np.ndarray:
    P = np.zeros((3, 4))
    P[:, :3] = R
    P[:, 3] = t
    return P.reshape(12).astype(np.float64)


# ---------------------------------------------------------------------------
# painting

def paint_ellipsoid(labels: np.ndarray, centre, semi, R, value: int) -> None:
    """Set voxels whose centre lies inside the rotated ellipsoid to `value`."""
    nz, ny, nx = labels.shape
    rad = float(max(semi)) + 1.0
    lo = [max(0, int(math.floor(centre[i] - rad))) for i in range(3)]
    hi = [min(n, int(math.ceil(centre[i] + rad)) + 1) for i, n in enumerate((nx, ny, nz))]
    if any(h <= l for l, h in zip(lo, hi)):
        return
    zz, yy, xx = np.meshgrid(
        np.arange(lo[2], hi[2]), np.arange(lo[1], hi[1]), np.arange(lo[0], hi[0]), indexing="ij"
    )
    d = np.stack([xx - centre[0], yy - centre[1], zz - centre[2]], axis=-1)  # (.., 3)
    local = d @ np.asarray(R)  # R^T d in row form
    q = (local[..., 0] / semi[0]) ** 2 + (local[..., 1] / semi[1]) ** 2 + (local[..., 2] / semi[2]) ** 2
    sub = labels[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
    sub[q <= 1.0] = value


def ellipsoid_volume(seed: int, n: int = 64, n_ellipsoids: int = 6) -> np.ndarray:
    """64^3 soft-tissue block with seeded fat/bone ellipsoids (painted in order)."""
    rng = np.random.default_rng(seed)
    lab = np.full((n, n, n), SOFT, dtype=np.uint8)
    s = n / 64.0
    for _ in range(n_ellipsoids):
        value = int(rng.integers(FAT, BONE + 1))
        centre = rng.uniform(12 * s, 52 * s, size=3)
        semi = rng.uniform(3 * s, 12 * s, size=3)
        paint_ellipsoid(lab, centre, semi, random_rotation(rng), value)
    return lab


def ct_from_labels(labels: np.ndarray, seed: int) -> np.ndarray:
    """int16 CT-like volume: HU ~ N(mean(label), 30), rounded, clamped."""
    rng = np.random.default_rng(seed ^ 0x5EED)
    mu = np.asarray(HU_MEAN, dtype=np.float32)[labels]
    hu = mu + rng.standard_normal(labels.shape, dtype=np.float32) * np.float32(HU_SD)
    return np.clip(np.rint(hu), -1024, 3071).astype(np.int16)


@dataclass
class BodyGeom:
    """Geometry of the spine-like phantom in voxel units (x, y, z)."""
    cx: float
    cz: float
    ax: float  # body semi-axis along x
    az: float  # body semi-axis along z (z large = back)

    def back_skin_z(self, x):
        u = np.clip((x - self.cx) / self.ax, -1.0, 1.0)
        return self.cz + self.az * np.sqrt(1.0 - u * u)


def spine_volume(dims, seed: int):
    """Body cylinder along y, fat layer under the back, 5 bone ellipsoids.

    dims = (nx, ny, nz).  Returns (labels uint8 [nz][ny][nx], BodyGeom).
    """
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    geom = BodyGeom(cx=nx / 2.0, cz=nz / 2.0, ax=0.43 * nx, az=0.31 * nz)
    x = np.arange(nx, dtype=np.float32)[None, :]
    z = np.arange(nz, dtype=np.float32)[:, None]
    q_out = ((x - geom.cx) / geom.ax) ** 2 + ((z - geom.cz) / geom.az) ** 2
    q_in = ((x - geom.cx) / (geom.ax - 10.0)) ** 2 + ((z - geom.cz) / (geom.az - 10.0)) ** 2
    sl = np.full((nz, nx), AIR, dtype=np.uint8)
    sl[q_out <= 1.0] = SOFT
    sl[(q_out <= 1.0) & (q_in > 1.0) & (z > geom.cz)] = FAT
    lab = np.ascontiguousarray(np.broadcast_to(sl[:, None, :], (nz, ny, nx)))
    spacing = 35.0 * ny / 256.0
    depth = 60.0
    zc = geom.cz + geom.az - depth
    for i in range(5):
        centre = (
            geom.cx + rng.uniform(-3, 3),
            ny / 2.0 + (i - 2) * spacing + rng.uniform(-3, 3),
            zc + rng.uniform(-3, 3),
        )
        semi = (20.0 * rng.uniform(0.9, 1.1), 12.0 * rng.uniform(0.9, 1.1), 15.0 * rng.uniform(0.9, 1.1))
        R = _rot_axis(1, rng.uniform(-0.15, 0.15)) @ _rot_axis(0, rng.uniform(-0.15, 0.15))
        paint_ellipsoid(lab, centre, semi, R, BONE)
    return lab, geom


def spine_pose(geom: BodyGeom, ny: int, rng: np.random.Generator, inset: float = 3.0) -> np.ndarray:
    """Probe on the back skin near the spine, beam into the body (-z),
    random rotation about the beam and tilts in [-20, 20] deg."""
    x0 = geom.cx + rng.uniform(-30, 30)
    y0 = ny / 2.0 + rng.uniform(-30, 30)
    z0 = float(geom.back_skin_z(x0)) - inset
    # base: probe x -> +x, probe z (beam) -> -z, probe y = z cross x -> -y
    base = np.array([[1.0, 0, 0], [0, -1.0, 0], [0, 0, -1.0]]).T
    R = (
        base
        @ _rot_axis(2, rng.uniform(0, 2 * math.pi))
        @ _rot_axis(0, math.radians(rng.uniform(-20, 20)))
        @ _rot_axis(1, math.radians(rng.uniform(-20, 20)))
    )
    return pose_from(R, (x0, y0, z0))


# ---------------------------------------------------------------------------
# workloads

def ellipsoid_workload(seed: int = 0, n_envs: int = 1, W: int = 64, H: int = 128,
                       dx: float = 0.5, dy: float = 0.5, n: int = 64) -> Workload:
    """Plain physics, 64^3 ellipsoid phantoms: one volume per env, pose origin
    ~U[16,48]^3 mm with a uniform random rotation."""
    vols, poses = [], []
    for e in range(n_envs):
        s = seed * 1000003 + e
        vols.append(Volume(labels=ellipsoid_volume(s, n=n), seed=(0x9E3779B97F4A7C15 * (s + 1)) & ((1 << 64) - 1)))
        rng = np.random.default_rng(s + 7919)
        t = rng.uniform(16 * n / 64, 48 * n / 64, size=3)
        poses.append(pose_from(random_rotation(rng), t))
    probes = [Probe(W=W, H=H, dx=dx, dy=dy) for _ in range(n_envs)]
    return Workload(vols, np.arange(n_envs, dtype=np.int32), probes, np.stack(poses))


def spine_ct_workload(seed: int = 0, n_envs: int = 64, dims=(256, 256, 256), W: int = 128, H: int = 256) -> Workload:
    """64 envs on one 256^3 spine phantom with an int16 CT volume."""
    lab, geom = spine_volume(dims, seed)
    ct = ct_from_labels(lab, seed)
    vol = Volume(labels=lab, ct=ct, seed=0xC0FFEE ^ (seed << 20))
    rng = np.random.default_rng(seed + 104729)
    poses = np.stack([spine_pose(geom, dims[1], rng) for _ in range(n_envs)])
    probes = [Probe(W=W, H=H) for _ in range(n_envs)]
    return Workload([vol], np.zeros(n_envs, dtype=np.int32), probes, poses)


def batched_dims(n_vols: int = 8, lo=(160, 160, 160), hi=(320, 256, 384)):
    out = []
    for v in range(n_vols):
        f = v / max(1, n_vols - 1)
        out.append(tuple(int(round(a + (b - a) * f)) for a, b in zip(lo, hi)))
    return out


def batched_workload(seed: int = 0, n_envs: int = 256, n_vols: int = 8,
                     W_range=(64, 256), H_range=(128, 512)) -> Workload:
    """Uneven batch: 8 label-only spine phantoms from 160^3 to 320x256x384,
    env e uses volume e mod 8, image size W ~ U{64..256}, H ~ U{128..512}."""
    vols, geoms = [], []
    for v, d in enumerate(batched_dims(n_vols)):
        lab, g = spine_volume(d, seed * 131 + v)
        vols.append(Volume(labels=lab, seed=(seed * 0x100000001B3 + 17 * v + 1) & ((1 << 64) - 1)))
        geoms.append((g, d))
    rng = np.random.default_rng(seed + 15485863)
    vol_ids = (np.arange(n_envs) % n_vols).astype(np.int32)
    probes, poses = [], []
    for e in range(n_envs):
        g, d = geoms[vol_ids[e]]
        W = int(rng.integers(W_range[0], W_range[1] + 1))
        H = int(rng.integers(H_range[0], H_range[1] + 1))
        probes.append(Probe(W=W, H=H))
        poses.append(spine_pose(g, d[1], rng))
    return Workload(vols, vol_ids, probes, np.stack(poses))


def volumetric_workload(seed: int = 0, n_envs: int = 256, n_vols: int = 8) -> Workload:
    """The uneven batch's volumes and probe poses with the surgery task's
    volumetric probe: 37 scanlines x 50 depth samples at 2 mm, 5 elevation
    planes 10 mm apart (H x W x E = 50 x 37 x 5 at 2 x 2 x 10 mm)."""
    wl = batched_workload(seed=seed, n_envs=n_envs, n_vols=n_vols)
    wl.probes = [Probe(W=37, H=50, dx=2.0, dy=2.0, n_elev=5, elev=10.0) for _ in range(n_envs)]
    return wl
