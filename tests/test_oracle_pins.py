"""Pins of the FP64 oracle against things other than itself: library
generators and routines, closed forms, brute force on tiny inputs,
invariants and published constants.  CPU only."""
from fractions import Fraction
from math import isqrt, sqrt

import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.stats as st

import oracle
import synth
from cases import axis_pose, layered_volume, single_env, table_with
from synth import Probe, Volume

M64 = (1 << 64) - 1


# ---------------------------------------------------------------------------
# O7: Philox

@pytest.mark.parametrize("key,ctr", [(0, 0), (1, 0), (0x0123456789ABCDEF_FEDCBA9876543210, 5),
                                     (12345, (1 << 64) - 1), (M64, (1 << 200) + 77)])
def test_philox4x64_round_structure_matches_numpy(key, ctr):
    """The shared round/key-schedule structure, instantiated at 64 bits,
    reproduces numpy's Philox (4x64-10).  numpy advances the 256-bit counter
    by one before producing each block of four words."""
    bg = np.random.Philox(key=key, counter=ctr)
    raw = bg.random_raw(12)
    kw = [(key >> (64 * i)) & M64 for i in range(2)]
    for blk in range(3):
        c = (ctr + 1 + blk) % (1 << 256)
        cw = [(c >> (64 * i)) & M64 for i in range(4)]
        got = oracle.philox4x64(cw, kw)
        assert [int(g) for g in got] == [int(r) for r in raw[4 * blk:4 * blk + 4]]


def test_philox4x32_constants():
    """One round exposes the multipliers, two rounds from zero expose the
    Weyl key increments.  Multipliers: Salmon et al. (SC'11); increments:
    first 32 fractional bits of the golden ratio and of sqrt(3)."""
    one = oracle.philox4x32([1, 0, 0, 0], [0, 0], rounds=1)
    assert int(one[3]) == 0xD2511F53 and int(one[2]) == 0
    one = oracle.philox4x32([0, 0, 1, 0], [0, 0], rounds=1)
    assert int(one[1]) == 0xCD9E8D57 and int(one[0]) == 0
    two = oracle.philox4x32([0, 0, 0, 0], [0, 0], rounds=2)
    w0 = (isqrt(5 << 64) - (1 << 32)) >> 1      # frac((1+sqrt5)/2) * 2^32
    w1 = isqrt(3 << 64) - (1 << 32)             # frac(sqrt3) * 2^32
    assert (int(two[0]), int(two[1]), int(two[2]), int(two[3])) == (w0, 0, w1, 0)
    # the 64-bit instantiation's increments, from the same definition
    two64 = oracle.philox4x64([0, 0, 0, 0], [0, 0], rounds=2)
    assert int(two64[0]) == (isqrt(5 << 128) - (1 << 64)) >> 1
    assert int(two64[2]) == isqrt(3 << 128) - (1 << 64)


def test_philox4x32_output_statistics():
    words = np.array([oracle.philox4x32([i, 0, 0, 0], [0xDEADBEEF, 7]) for i in range(20000)],
                     dtype=np.uint64)
    for lane in range(4):
        u = words[:, lane].astype(np.float64) / 2.0 ** 32
        assert abs(u.mean() - 0.5) < 4 * sqrt(1 / 12 / len(u))
        h, _ = np.histogram(u, bins=16, range=(0, 1))
        assert st.chisquare(h).pvalue > 1e-4
    # bits of neighbouring counters decorrelated
    c = np.corrcoef(words[:-1, 0].astype(np.float64), words[1:, 0].astype(np.float64))[0, 1]
    assert abs(c) < 0.04


def test_gate_threshold_matches_normal_cdf():
    for mu in [-3.0, -0.5, 0.0, 0.3, 0.5, 1.7, 4.0]:
        m = float(np.float32(mu))
        assert oracle.gate_threshold(m) == int(np.floor(st.norm.cdf(m) * 2.0 ** 32))
    assert oracle.gate_threshold(float("-inf")) == 0
    assert oracle.gate_threshold(float("inf")) == 1 << 32


def _noise_slab(n=256, sigma0=1.0, mu0=0.0, mu1=np.inf, seed=99):
    vol = Volume(labels=np.ones((n, 1, n), dtype=np.uint8), seed=seed)
    probe = Probe(W=n, H=n, dx=1.0, dy=1.0)
    table = table_with(sigma0_1=sigma0, mu0_1=mu0, mu1_1=mu1)
    return oracle.simulate_env(vol, table, probe, axis_pose(((n - 1) / 2.0, 0.0, 0.0)),
                               planes=("T", "voxel", "philox"))


def test_box_muller_is_standard_normal():
    o = _noise_slab()
    assert (o["voxel"] >= 0).all() and len(np.unique(o["voxel"])) == o["voxel"].size
    n0 = o["T"].ravel()
    n = n0.size
    assert abs(n0.mean()) < 4 / sqrt(n)
    assert abs(n0.var() - 1.0) < 4 * sqrt(2.0 / n)
    assert st.kstest(n0, "norm").pvalue > 1e-4


def test_gate_fraction_is_phi_mu1():
    o = _noise_slab(sigma0=0.0, mu0=1.0, mu1=0.3)
    frac = (o["T"] == 1.0).mean()
    p = st.norm.cdf(float(np.float32(0.3)))
    assert abs(frac - p) < 4 * sqrt(p * (1 - p) / o["T"].size)


def test_noise_is_keyed_by_voxel():
    rng = np.random.default_rng(3)
    vol = Volume(labels=rng.integers(1, 4, size=(12, 10, 14)).astype(np.uint8), seed=0xABCDEF0123)
    probe = Probe(W=17, H=23, dx=0.37, dy=0.41)
    pose = synth.pose_from(synth.random_rotation(rng), (6.5, 5.1, 4.2))
    o = oracle.simulate_env(vol, synth.default_tissue_table(), probe, pose, planes=("voxel", "philox"))
    key = [0xABCDEF0123 & 0xFFFFFFFF, 0xABCDEF0123 >> 32]
    inside = o["voxel"] >= 0
    assert inside.sum() > 20 and (~inside).sum() > 0
    for yy, xx in zip(*np.nonzero(inside)):
        n = int(o["voxel"][yy, xx])
        assert list(o["philox"][yy, xx]) == list(oracle.philox4x32([n, 0, 0, 0], key))
    assert (o["philox"][~inside] == 0).all()


# ---------------------------------------------------------------------------
# O1, O2: geometry and nearest-label sampling

def _rand_labels(shape, seed):
    return np.random.default_rng(seed).integers(0, 4, size=shape).astype(np.uint8)


def test_axis_aligned_slice_equals_numpy_slice():
    lab = _rand_labels((20, 7, 24), 5)
    vol = Volume(labels=lab, seed=1)
    probe = Probe(W=9, H=30, dx=1.0, dy=1.0)
    t = (10.0, 3.0, -2.0)   # pixel (x, y) -> voxel (6 + x, 3, -2 + y)
    o = oracle.simulate_env(vol, synth.default_tissue_table(), probe, axis_pose(t),
                            planes=("label", "voxel"))
    for y in range(30):
        for x in range(9):
            ix, iy, iz = 6 + x, 3, -2 + y
            if 0 <= iz < 20:
                assert o["label"][y, x] == lab[iz, iy, ix]
                assert o["voxel"][y, x] == (iz * 7 + iy) * 24 + ix
            else:
                assert o["label"][y, x] == 0 and o["voxel"][y, x] == -1


def test_rotated_slice_equals_transposed_numpy_slice():
    lab = _rand_labels((9, 20, 16), 6)
    vol = Volume(labels=lab, spacing=(0.5, 1.0, 2.0), seed=1)
    # probe x -> volume y, probe z (beam) -> volume x, probe y -> volume z
    R = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    probe = Probe(W=11, H=10, dx=1.0, dy=0.5)
    t = (0.0, 8.0, 8.0)   # voxel coords: x = y*0.5/0.5, y = 3 + x, z = 4
    o = oracle.simulate_env(vol, synth.default_tissue_table(), probe, axis_pose(t, R),
                            planes=("label",))
    expect = np.zeros((10, 11), dtype=np.uint8)
    for y in range(10):
        for x in range(11):
            ix, iy, iz = y, 3 + x, 4
            if ix < 16 and iy < 20:
                expect[y, x] = lab[iz, iy, ix]
    assert (o["label"] == expect).all()


def test_q16_geometry_within_rounding_bound():
    rng = np.random.default_rng(11)
    for trial in range(20):
        sp = tuple(rng.uniform(0.3, 2.0, size=3))
        vol = Volume(labels=np.ones((4, 4, 4), dtype=np.uint8), spacing=sp)
        probe = Probe(W=int(rng.integers(1, 300)), H=int(rng.integers(1, 600)),
                      dx=float(rng.uniform(0.1, 1)), dy=float(rng.uniform(0.1, 1)))
        pose = synth.pose_from(synth.random_rotation(rng), rng.uniform(-50, 250, size=3))
        P0, DX, DY = oracle.geometry(vol, probe, pose)
        R = pose.reshape(3, 4)[:, :3]
        t = pose.reshape(3, 4)[:, 3]
        for (x, y) in [(0, 0), (probe.W - 1, 0), (0, probe.H - 1), (probe.W - 1, probe.H - 1)]:
            pp = np.array([-0.5 * (probe.W - 1) * probe.dx + x * probe.dx, 0.0, y * probe.dy])
            exact = (R @ pp + t) / np.array(sp)
            q = (P0 + x * DX + y * DY) / 65536.0
            assert np.all(np.abs(q - exact) <= (0.5 + 0.5 * x + 0.5 * y) / 65536.0 + 1e-9)


def test_nearest_label_brute_force_tiny():
    """Argmin over all voxel centres of the exact rational position."""
    rng = np.random.default_rng(21)
    for trial in range(6):
        shape = (4, 5, 6)
        lab = _rand_labels(shape, 100 + trial)
        sp = (1.0, 0.75, 1.25) if trial % 2 else (1.0, 1.0, 1.0)
        vol = Volume(labels=lab, spacing=sp, seed=3)
        probe = Probe(W=5, H=7, dx=0.8, dy=0.6)
        pose = synth.pose_from(synth.random_rotation(rng), rng.uniform(0.5, 4.0, size=3))
        o = oracle.simulate_env(vol, synth.default_tissue_table(), probe, pose,
                                planes=("q", "label", "voxel"))
        nz, ny, nx = shape
        for y in range(probe.H):
            for x in range(probe.W):
                q = [Fraction(int(v), 65536) for v in o["q"][y, x]]
                inside = all(Fraction(-1, 2) <= q[c] < Fraction(n, 1) - Fraction(1, 2)
                             for c, n in enumerate((nx, ny, nz)))
                if not inside:
                    assert o["label"][y, x] == 0 and o["voxel"][y, x] == -1
                    continue
                best, arg = None, None
                for iz in range(nz):
                    for iy in range(ny):
                        for ix in range(nx):
                            d = (q[0] - ix) ** 2 + (q[1] - iy) ** 2 + (q[2] - iz) ** 2
                            # ties go to the larger index (half-up rounding)
                            if best is None or d <= best:
                                best, arg = d, (ix, iy, iz)
                ix, iy, iz = arg
                assert o["voxel"][y, x] == (iz * ny + iy) * nx + ix
                assert o["label"][y, x] == lab[iz, iy, ix]


# ---------------------------------------------------------------------------
# O3: CT trilinear

def test_ct_trilinear_matches_scipy():
    rng = np.random.default_rng(8)
    lab = np.ones((10, 12, 14), dtype=np.uint8)
    ct = rng.integers(-1024, 2000, size=lab.shape).astype(np.int16)
    vol = Volume(labels=lab, ct=ct, spacing=(1.0, 0.9, 1.1), seed=4)
    probe = Probe(W=33, H=41, dx=0.37, dy=0.29)
    pose = synth.pose_from(synth.random_rotation(rng), (7.0, 5.0, 5.5))
    o = oracle.simulate_env(vol, synth.default_tissue_table(), probe, pose, planes=("q", "Z"))
    q = o["q"].reshape(-1, 3).astype(np.float64) / 65536.0
    hu = ndi.map_coordinates(ct.astype(np.float64), [q[:, 2], q[:, 1], q[:, 0]], order=1,
                             mode="grid-constant", cval=-1000.0)
    Z = np.maximum(hu + 1000.0, 0.0).reshape(probe.H, probe.W)
    assert np.allclose(o["Z"], Z, rtol=1e-12, atol=1e-9)
    assert (o["Z"] == 0).any() and (o["Z"] > 0).any()


# ---------------------------------------------------------------------------
# O4: reflection / transmission

def _interface_run(table=None, ct=False, seed=12):
    rng = np.random.default_rng(seed)
    lab = rng.integers(0, 4, size=(16, 16, 16)).astype(np.uint8)
    vol = Volume(labels=lab, ct=synth.ct_from_labels(lab, seed) if ct else None, seed=5)
    probe = Probe(W=21, H=40, dx=0.5, dy=0.5)
    pose = synth.pose_from(synth.random_rotation(rng), (8.0, 8.0, 8.0))
    return oracle.simulate_env(vol, synth.default_tissue_table() if table is None else table,
                               probe, pose, planes=("label", "G", "r", "t", "Z", "Y"))


@pytest.mark.parametrize("ct", [False, True])
def test_reflection_transmission_invariants(ct):
    o = _interface_run(ct=ct)
    r, t, G = o["r"], o["t"], o["G"].astype(bool)
    assert G.sum() > 10
    assert np.allclose(r * r + t, 1.0, atol=1e-12)
    assert (np.abs(r) <= 1.0).all() and (t >= 0).all() and (t <= 1).all()
    assert (r[~G] == 0).all() and (t[~G] == 1).all()
    # G is exactly "label changes between y and y+1"
    lab = o["label"].astype(int)
    assert (G[:-1] == (lab[:-1] != lab[1:])).all() and not G[-1].any()


def test_reflection_scale_invariance():
    base = synth.default_tissue_table()
    scaled = base.copy()
    scaled[:, 0] *= 4.0   # exact power-of-two scale of every impedance
    a, b = _interface_run(base), _interface_run(scaled)
    assert np.array_equal(a["r"], b["r"]) and np.array_equal(a["t"], b["t"])
    assert np.array_equal(a["Y"], b["Y"])


# ---------------------------------------------------------------------------
# O5: energy closed forms

def _slab_env(layers, table, H=120, W=15, dy=0.5, E0=1.0, n=64):
    vol = layered_volume(n, n, n, layers)
    probe = Probe(W=W, H=H, dx=0.5, dy=dy, E0=E0)
    # beam along +z from z = 0, centred laterally
    return vol, probe, axis_pose((n / 2.0, n / 2.0, 0.0)), table


def test_energy_homogeneous_slab_closed_form():
    table = synth.default_tissue_table()
    vol, probe, pose, _ = _slab_env([(0, 1)], table, H=70)
    o = oracle.simulate_env(vol, table, probe, pose, planes=("E",))
    y = np.arange(probe.H)[:, None]
    alpha = float(table[1, 1])
    expect = probe.E0 * np.exp(-probe.f * alpha * y * probe.dy / 10.0)
    assert np.allclose(o["E"], np.broadcast_to(expect, o["E"].shape), rtol=1e-12, atol=0)


def test_energy_two_interfaces_closed_form():
    table = synth.default_tissue_table()
    # soft voxels 0..9, fat 10..19, soft 20..; row v samples voxel round_half_up(v/2),
    # so the boundary rows (G = 1) are 18 and 38
    vol, probe, pose, _ = _slab_env([(0, 1), (10, 2), (20, 1)], table, H=70, E0=2.5)
    o = oracle.simulate_env(vol, table, probe, pose, planes=("E", "label"))
    Z1, Z2 = float(table[1, 0]), float(table[2, 0])
    r = (Z2 - Z1) / (Z2 + Z1)
    t = 1.0 - r * r
    a = {l: float(table[l, 1]) for l in (1, 2)}
    E = []
    for y in range(probe.H):
        # labels along the path before y: rows v < y, row v at z = v * dy
        path = [1 if (v + 1) // 2 < 10 else (2 if (v + 1) // 2 < 20 else 1) for v in range(y)]
        n_int = sum(1 for v in range(y) if v in (18, 38))
        E.append(2.5 * t ** n_int * np.exp(-probe.f * probe.dy / 10.0 * sum(a[l] for l in path)))
    assert np.allclose(o["E"], np.array(E)[:, None], rtol=1e-12, atol=0)


@pytest.mark.parametrize("Zb", [np.inf, 0.0])
def test_total_reflection_single_bone_interface(Zb):
    """Bone layer with infinite (or zero) impedance: nothing is transmitted,
    so E and the scattering term vanish below the interface and I is exactly
    zero farther than the axial PSF radius below it."""
    table = table_with(Z_3=Zb)
    vol, probe, pose, _ = _slab_env([(0, 1), (15, 3)], table, H=120)
    o = oracle.simulate_env(vol, table, probe, pose, planes=("E", "I", "Rp", "G", "r"))
    yb = 28   # last soft-tissue row (z = 14 mm; row 29 at 14.5 mm rounds up into bone)
    assert o["G"][yb].all() and (np.abs(o["r"][yb]) == 1.0).all()
    assert (o["E"][yb + 1:] == 0).all() and (o["E"][:yb + 1] > 0).all()
    rax = (len(oracle.psf_kernel(0.01 * probe.H)) - 1) // 2
    assert (o["I"][yb + rax + 1:] == 0).all()
    assert (o["I"][yb] > 0).all()


# ---------------------------------------------------------------------------
# O6: incidence angle

def test_cos_theta_horizontal_interface_is_one():
    table = synth.default_tissue_table()
    vol, probe, pose, _ = _slab_env([(0, 1), (15, 3)], table, H=60)
    o = oracle.simulate_env(vol, table, probe, pose, planes=("G", "cos_theta"))
    assert o["G"].sum() == probe.W and (o["cos_theta"] == 1.0).all()


def test_cos_theta_45_degree_staircase():
    n = 40
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    lab = np.where(xx + zz < 40, 1, 3).astype(np.uint8)
    vol = Volume(labels=lab, seed=2)
    probe = Probe(W=21, H=30, dx=1.0, dy=1.0)
    pose = axis_pose((20.0, 20.0, 0.0))    # pixel (x, y) -> voxel (10 + x, 20, y)
    o = oracle.simulate_env(vol, synth.default_tissue_table(), probe, pose, planes=("G", "cos_theta"))
    ys, xs = np.nonzero(o["G"])
    interior = (xs > 0) & (xs < probe.W - 1) & (ys > 0)
    assert interior.sum() > 10
    assert np.allclose(o["cos_theta"][ys[interior], xs[interior]], 1 / sqrt(2), rtol=1e-15)


@pytest.mark.parametrize("dx,dy", [(1.0, 0.5), (0.5, 1.0), (0.37, 0.29)])
def test_cos_theta_pixel_diagonal_with_anisotropic_pixels(dx, dy):
    """Labels split on ix + iz, imaged by an axis-aligned plane whose pixels
    are the voxels (pitch dx laterally, dy axially): the interface runs along
    the pixel diagonals, i.e. along the physical direction (dx, -dy), so its
    normal is (dy, dx) / |(dx, dy)| and the beam (axial) meets it at
    cos(theta) = dx / sqrt(dx^2 + dy^2).  Swapping the physical scaling of
    the two Sobel sums would give dy / sqrt(dx^2 + dy^2) instead."""
    n = 40
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    lab = np.where(xx + zz < 40, 1, 3).astype(np.uint8)
    vol = Volume(labels=lab, spacing=(dx, 1.0, dy), seed=2)
    probe = Probe(W=21, H=30, dx=dx, dy=dy)
    # pixel (x, y) -> probe point ((x - 10) dx, 0, y dy) -> voxel (10 + x, 20, y)
    pose = axis_pose((20.0 * dx, 20.0, 0.0))
    g = oracle.geometry(vol, probe, pose)
    assert [int(v) for v in g[0]] == [10 << 16, 20 << 16, 0] and [int(v) for v in g[1]] == [1 << 16, 0, 0]
    assert [int(v) for v in g[2]] == [0, 0, 1 << 16]
    o = oracle.simulate_env(vol, synth.default_tissue_table(), probe, pose, planes=("G", "cos_theta", "label"))
    assert np.array_equal(o["label"], np.where(10 + np.arange(21)[None, :] + np.arange(30)[:, None] < 40, 1, 3))
    ys, xs = np.nonzero(o["G"])
    interior = (xs > 0) & (xs < probe.W - 1) & (ys > 0)
    assert interior.sum() > 10
    want = dx / sqrt(dx * dx + dy * dy)
    assert np.allclose(o["cos_theta"][ys[interior], xs[interior]], want, rtol=1e-15, atol=0)


# ---------------------------------------------------------------------------
# O9 .. O11

def test_psf_kernel_is_normalised_sampled_gaussian():
    for sigma in [0.01, 0.64, 1.28, 2.56, 5.12]:
        K = oracle.psf_kernel(sigma)
        r = (len(K) - 1) // 2
        assert r == max(1, int(np.ceil(3 * sigma)))
        k = np.arange(-r, r + 1)
        g = st.norm.pdf(k, scale=sigma)
        assert np.allclose(K, g / g.sum(), rtol=1e-12)


def test_composition_matches_scipy_separable_convolution():
    wl = synth.ellipsoid_workload(seed=4, n_envs=1, W=48, H=96)
    p = wl.probes[0]
    o = oracle.simulate_env(wl.volumes[0], wl.table, p, wl.poses[0],
                            planes=("Rp", "T", "E", "I", "A"))
    Kax, Klat = oracle.psf_kernel(0.01 * p.H), oracle.psf_kernel(0.01 * p.W)

    def conv(f):
        g = ndi.correlate1d(f, Kax, axis=0, mode="constant", cval=0.0)
        return ndi.correlate1d(g, Klat, axis=1, mode="constant", cval=0.0)

    I = conv(o["Rp"]) + o["E"] * conv(o["T"])
    A = conv(o["Rp"]) + o["E"] * conv(np.abs(o["T"]))
    assert np.allclose(o["I"], I, rtol=0, atol=1e-13 * max(1.0, A.max()))
    assert np.allclose(o["A"], A, rtol=1e-12, atol=1e-300)
    assert (o["Rp"] > 0).any() and (o["T"] != 0).any()


def test_slab_intensity_closed_form_and_display():
    table = table_with(sigma0_1=0.0, mu1_1=np.inf, mu0_1=0.05)
    vol, probe, pose, _ = _slab_env([(0, 1)], table, H=100, W=31)
    o = oracle.simulate_env(vol, table, probe, pose, planes=("I", "Y"))
    rax = (len(oracle.psf_kernel(0.01 * probe.H)) - 1) // 2
    rlat = (len(oracle.psf_kernel(0.01 * probe.W)) - 1) // 2
    y = np.arange(rax, probe.H - rax)[:, None]
    expect = 0.05 * probe.E0 * np.exp(-probe.f * float(table[1, 1]) * y * probe.dy / 10.0)
    inner = o["I"][rax:probe.H - rax, rlat:probe.W - rlat]
    assert np.allclose(inner, np.broadcast_to(expect, inner.shape), rtol=1e-12)
    # display: dB map with 60 dB range anchored at E0
    Yi = o["Y"][rax:probe.H - rax, rlat:probe.W - rlat]
    dYdy = np.diff(Yi[:, 0])
    slope = (20.0 / probe.dr) * (-probe.f * float(table[1, 1]) * probe.dy / 10.0) / np.log(10.0)
    assert np.allclose(dYdy, slope, rtol=1e-9)
    assert np.allclose(Yi[0, 0], 1.0 + (20.0 / 60.0) * np.log10(expect[0, 0]), rtol=1e-12)


def test_single_interface_reflection_closed_form():
    table = table_with(sigma0_1=0.0, mu0_1=0.0, sigma0_2=0.0, mu0_2=0.0)
    vol, probe, pose, _ = _slab_env([(0, 1), (15, 2)], table, H=100, W=31)
    o = oracle.simulate_env(vol, table, probe, pose, planes=("I", "E"))
    yb = 28   # last row of layer 1
    Z1, Z2 = float(table[1, 0]), float(table[2, 0])
    r = abs((Z2 - Z1) / (Z2 + Z1))
    Kax = oracle.psf_kernel(0.01 * probe.H)
    rax = (len(Kax) - 1) // 2
    rlat = (len(oracle.psf_kernel(0.01 * probe.W)) - 1) // 2
    Eb = o["E"][yb, 0]
    for y in range(probe.H):
        j = y - yb
        expect = Eb * r * Kax[j + rax] if abs(j) <= rax else 0.0
        assert np.allclose(o["I"][y, rlat:probe.W - rlat], expect, rtol=1e-12, atol=0)


def test_intensity_linear_in_E0_and_display_anchor():
    wl = synth.ellipsoid_workload(seed=2, n_envs=1)
    p1 = wl.probes[0]
    p2 = Probe(**{**p1.__dict__, "E0": 4.0})
    a = oracle.simulate_env(wl.volumes[0], wl.table, p1, wl.poses[0], planes=("I", "Y"))
    b = oracle.simulate_env(wl.volumes[0], wl.table, p2, wl.poses[0], planes=("I", "Y"))
    assert np.allclose(b["I"], 4.0 * a["I"], rtol=1e-12, atol=1e-300)
    assert np.allclose(a["Y"], b["Y"], atol=1e-12)


def test_label_permutation_invariance():
    wl = synth.ellipsoid_workload(seed=3, n_envs=1)
    perm = np.array([0, 3, 1, 2], dtype=np.uint8)   # keep air as label 0
    vol = wl.volumes[0]
    vol2 = Volume(labels=perm[vol.labels], seed=vol.seed)
    table2 = np.zeros_like(wl.table)
    table2[perm] = wl.table
    a = oracle.simulate_env(vol, wl.table, wl.probes[0], wl.poses[0], planes=("I", "Y"))
    b = oracle.simulate_env(vol2, table2, wl.probes[0], wl.poses[0], planes=("I", "Y"))
    assert np.array_equal(a["I"], b["I"]) and np.array_equal(a["Y"], b["Y"])


def test_batch_equals_single_env_and_is_deterministic():
    wl = synth.ellipsoid_workload(seed=5, n_envs=3, W=40, H=70)
    frames, used = oracle.simulate_batch(wl, n_threads=2)
    for e in range(3):
        o = oracle.simulate_env(wl.volumes[wl.vol_ids[e]], wl.table, wl.probes[e], wl.poses[e],
                                planes=("Y",))
        assert np.array_equal(frames[e], o["Y"])
    frames2, _ = oracle.simulate_batch(wl, n_threads=1)
    assert all(np.array_equal(a, b) for a, b in zip(frames, frames2))


def test_rejects_label_outside_table():
    vol = Volume(labels=np.full((4, 4, 4), 7, dtype=np.uint8))
    with pytest.raises(ValueError):
        oracle.simulate_env(vol, synth.default_tissue_table(), Probe(W=3, H=3),
                            axis_pose((2.0, 2.0, 1.0)))


# ---------------------------------------------------------------------------
# multi-scale noise (reading of the last sentence on the scattering pattern)

def test_quantised_normal_table_inverts_the_normal_cdf():
    """Q[k] is the quantile of (k + 1/2)/4096 rounded to a multiple of 2^-20:
    pinned by the forward CDF (a different library routine) bracketing the
    probability between the half-steps around Q, odd symmetry and
    monotonicity."""
    from scipy.stats import norm
    q = oracle.quantised_normal_table()
    assert q.dtype == np.int32 and q.shape == (4096,)
    p = (np.arange(4096) + 0.5) / 4096.0
    lo = norm.cdf((q.astype(np.float64) - 0.5) * 2.0 ** -20)
    hi = norm.cdf((q.astype(np.float64) + 0.5) * 2.0 ** -20)
    assert np.all(lo <= p) and np.all(p <= hi)
    assert np.array_equal(q, -q[::-1]) and np.all(np.diff(q) > 0)
    # next to the median Phi^-1(1/2 + e) = sqrt(2 pi) e + O(e^3): the entry
    # above the median is rint(sqrt(2 pi) 2^-13 2^20)
    assert q[2048] == round(sqrt(2 * np.pi) * 2.0 ** -13 * 2.0 ** 20) == 321


def test_multiscale_threshold_is_the_exact_floor():
    """floor(sqrt(S) mu1 2^20) against exact rational arithmetic: n <= sqrt(S)
    mu1 2^20 is decided on squares of exact rationals (mu1 as its FP32 value),
    and the threshold is the largest such integer n."""
    def exact_floor(S, mu1):
        m = Fraction(float(np.float32(mu1))) * (1 << 20)
        # largest integer n with n <= sqrt(S) * m
        if m >= 0:
            n = isqrt(int(S * m * m))          # candidate for sqrt(S m^2)
            while (n + 1) ** 2 <= S * m * m:
                n += 1
            while n * n > S * m * m:
                n -= 1
            return n
        # m < 0: n <= -sqrt(S m^2)  <=>  n <= -ceil(sqrt(S m^2))
        c = isqrt(int(S * m * m))
        while c * c < S * m * m:
            c += 1
        return -c
    rng = np.random.default_rng(12)
    mus = [0.0, 0.5, -0.5, 1e-6, -1e-6, 0.3, 2.9, -2.9] + list(rng.normal(0, 1.5, 200))
    for S in (2, 3, 4):
        for mu in mus:
            assert oracle.multiscale_threshold(S, mu) == exact_floor(S, mu), (S, mu)
    assert oracle.multiscale_threshold(3, float("-inf")) == -(1 << 31)
    assert oracle.multiscale_threshold(3, float("inf")) == (1 << 31) - 1


def test_multiscale_gate_brute_force():
    """The gate of every voxel of a small multi-scale grid, recomputed from
    the generator's words (pinned against numpy's Philox above), the table and
    the exact-rational threshold: sum_s Q[w2_s >> 20] <= sqrt(S) mu1 2^20."""
    vol = _ms_volume(6, 3)
    q = oracle.quantised_normal_table()
    key = [41, 0]
    for mu1 in (0.4, -0.7):
        _, n1, g = oracle.scatter_grid(vol, mu1)
        m = Fraction(float(np.float32(mu1))) * (1 << 20)
        for iz in range(6):
            for iy in range(6):
                for ix in range(6):
                    tot = 0
                    for s in range(3):
                        mx = (6 + (1 << s) - 1) >> s
                        cell = ((iz >> s) * mx + (iy >> s)) * mx + (ix >> s)
                        tot += int(q[int(oracle.philox4x32([cell, 0, s, 0], key)[2]) >> 20])
                    assert int(n1[iz, iy, ix]) == tot
                    # tot <= sqrt(3) m, decided on exact squares
                    want = (tot <= 0 and (m >= 0 or tot * tot >= 3 * m * m)) or (tot > 0 and m > 0 and
                                                                                 tot * tot <= 3 * m * m)
                    assert bool(g[iz, iy, ix]) == want, (ix, iy, iz, tot)


def _ms_volume(n, scales, seed=41):
    return synth.Volume(labels=np.ones((n, n, n), np.uint8), seed=seed, noise_scales=scales)


def test_multiscale_scale_zero_is_the_voxel_stream():
    """Scale 0 of a multi-scale field draws the single-scale counters, and one
    scale is exactly the single-scale model."""
    v1, v3 = _ms_volume(16, 1), _ms_volume(16, 3)
    for ix, iy, iz in [(0, 0, 0), (5, 9, 13), (15, 15, 15)]:
        a = oracle.scatter_voxel(v1, 0.3, ix, iy, iz)
        b = oracle.scatter_voxel(v3, 0.3, ix, iy, iz)
        vox = (iz * 16 + iy) * 16 + ix
        assert np.array_equal(a[3], oracle.philox4x32([vox, 0, 0, 0], [41, 0]))
        assert np.array_equal(a[3], b[3])
        assert a[1] == 0.0 and a[2] == (int(a[3][2]) < oracle.gate_threshold(0.3))


@pytest.mark.parametrize("scales", [2, 3])
def test_multiscale_noise_statistics(scales):
    """N0 stays standard normal, the gate passes with probability Phi(mu1),
    and two voxels are correlated by the fraction of scales whose cell they
    share (1/S per shared scale): pins of the sum, its 1/sqrt(S) weight, the
    sqrt(S) threshold and the cell indexing."""
    from scipy.stats import norm
    vol = _ms_volume(64, scales)
    n0, n1, g = oracle.scatter_grid(vol, 0.5)
    assert abs(n0.mean()) < 0.03 and abs(n0.var() - 1.0) < 0.03
    assert abs(g.mean() - norm.cdf(0.5)) < 0.02
    for mu1 in (-0.5, 0.0):
        _, _, gm = oracle.scatter_grid(vol, mu1)
        assert abs(gm.mean() - norm.cdf(mu1)) < 0.02
    # neighbours along x: x = 4i + j and x + 1 share the cells of scales s
    # with (x >> s) == ((x + 1) >> s)
    for j in range(3):
        a = n0[:, :, j::4].ravel()
        b = n0[:, :, j + 1::4].ravel()
        shared = sum(1 for s in range(scales) if (j >> s) == ((j + 1) >> s))
        assert abs(np.corrcoef(a, b)[0, 1] - shared / scales) < 0.03, (j, shared)
    # N1 sums S unit-variance quantised normals: mean 0, variance S
    n1 = n1 * 2.0 ** -20
    assert abs(n1.mean()) < 0.05 * np.sqrt(scales) and abs(n1.var() / scales - 1.0) < 0.05


# ---------------------------------------------------------------------------
# volumetric probe: a stack of elevation planes (Sec. 4, surgery task)

def test_volumetric_planes_are_numpy_slices_at_their_elevation():
    """Axis-aligned probe with 5 planes 2 mm apart: plane j samples volume row
    y = 3 + (j - 2) * 2 (probe y -> volume y), each a numpy slice."""
    lab = _rand_labels((20, 13, 24), 8)
    vol = Volume(labels=lab, seed=1)
    probe = Probe(W=9, H=30, dx=1.0, dy=1.0, n_elev=5, elev=2.0)
    o = oracle.simulate_env(vol, synth.default_tissue_table(), probe, axis_pose((10.0, 7.0, -2.0)),
                            planes=("label", "voxel"))
    assert o["label"].shape == (5, 30, 9)
    for j in range(5):
        iy = 7 + (j - 2) * 2
        for y in range(30):
            iz = -2 + y
            for x in range(9):
                ix = 6 + x
                if 0 <= iz < 20:
                    assert o["label"][j, y, x] == lab[iz, iy, ix]
                    assert o["voxel"][j, y, x] == (iz * 13 + iy) * 24 + ix
                else:
                    assert o["label"][j, y, x] == 0


def test_volumetric_centre_plane_is_the_linear_probe():
    """An odd stack's centre plane has elevation 0 and is the linear probe's
    image bit for bit; the other planes follow the rotated elevation axis."""
    rng = np.random.default_rng(4)
    vol = Volume(labels=synth.ellipsoid_volume(3), seed=9)
    pose = synth.pose_from(synth.random_rotation(rng), (32.0, 30.0, 28.0))
    lin = Probe(W=20, H=40)
    vol3 = Probe(W=20, H=40, n_elev=3, elev=4.0)
    a = oracle.simulate_env(vol, synth.default_tissue_table(), lin, pose, planes=("q", "label", "Y"))
    b = oracle.simulate_env(vol, synth.default_tissue_table(), vol3, pose, planes=("q", "label", "Y"))
    assert np.array_equal(b["q"][1], a["q"]) and np.array_equal(b["Y"][1], a["Y"])
    # plane origins step by R (0, 4, 0) mm (in voxel Q16 units, within rounding)
    R = pose.reshape(3, 4)[:, :3]
    step = R @ np.array([0.0, 4.0, 0.0]) * 65536.0
    for j in (0, 2):
        d = (b["q"][j, 0, 0] - b["q"][1, 0, 0]).astype(np.float64)
        assert np.all(np.abs(d - (j - 1) * step) <= 1.0)


# ---------------------------------------------------------------------------
# reconstruction observation (bone-surface task)

def test_recon_surface_points_of_a_bone_slab_closed_form():
    """Bone (label 3) below z = 20 mm under soft tissue: every scanline's
    first bone pixel is row 20 (1 mm pixels from z = 0), so without misses the
    points lie at (x0 + a + x, y0, 20) mm."""
    vol = layered_volume(64, 64, 64, [(0, 1), (20, 3), (40, 1)])
    probe = Probe(W=31, H=50, dx=1.0, dy=1.0)
    pts = oracle.recon_points(vol, probe, axis_pose((32.0, 30.0, 0.0)), env=0, step=0, seed=5, p_drop=0.0)
    assert pts.shape == (31, 3)
    a = -0.5 * 30
    assert np.array_equal(pts[:, 0], 32.0 + a + np.arange(31.0))
    assert np.all(pts[:, 1] == 30.0) and np.all(pts[:, 2] == 20.0)
    # no bone in the image: no points
    assert oracle.recon_points(vol, Probe(W=8, H=15), axis_pose((32.0, 30.0, 0.0)), 0, 0, 5, 0.0).shape == (0, 3)


def test_recon_misses_points_with_the_stated_probability():
    vol = layered_volume(64, 64, 64, [(0, 1), (10, 3)])
    probe = Probe(W=1024, H=30, dx=0.05, dy=1.0)
    kept = [oracle.recon_points(vol, probe, axis_pose((32.0, 32.0, 0.0)), env=e, step=s, seed=9).shape[0]
            for e in range(4) for s in range(5)]
    frac = np.sum(kept) / (1024.0 * 20)
    assert abs(frac - 0.8) < 4 * np.sqrt(0.16 / (1024 * 20))
    a = oracle.recon_points(vol, probe, axis_pose((32.0, 32.0, 0.0)), env=1, step=2, seed=9)
    b = oracle.recon_points(vol, probe, axis_pose((32.0, 32.0, 0.0)), env=1, step=2, seed=9)
    c = oracle.recon_points(vol, probe, axis_pose((32.0, 32.0, 0.0)), env=1, step=3, seed=9)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_recon_observation_cells_closed_form():
    """Probe frame = volume frame shifted by t: a point at probe-frame (u_x,
    u_y, u_z) occupies cell (floor(u_z/3), floor((u_x+60)/3), floor((u_y+60)/3));
    points outside the 120 mm cube leave the grid empty."""
    t = np.array([10.0, -4.0, 7.0])
    pose = axis_pose(tuple(t))
    u = np.array([[0.0, 0.0, 0.0], [-59.9, 59.9, 119.9], [1.5, -1.5, 4.5], [0.0, 0.0, 120.0], [-60.1, 0.0, 3.0],
                  [0.0, 0.0, -0.1]])
    g = oracle.recon_observe(u + t, pose)
    expect = np.zeros((40, 40, 40), dtype=np.uint8)
    for ux, uy, uz in u[:3]:
        expect[int(np.floor(uz / 3)), int(np.floor((ux + 60) / 3)), int(np.floor((uy + 60) / 3))] = 1
    assert np.array_equal(g, expect) and g.sum() == 3
    # a rotated probe: points acquired and observed at the same pose land at
    # their pixel's depth and lateral cells; the image plane (elevation 0 up
    # to rounding) lies on the boundary of elevation cells 19 and 20
    rng = np.random.default_rng(2)
    vol = layered_volume(64, 64, 64, [(0, 1), (20, 3)])
    R = synth.random_rotation(rng)
    pose = synth.pose_from(R, (32.0, 32.0, 0.0))
    probe = Probe(W=40, H=60, dx=1.0, dy=1.0)
    pts = oracle.recon_points(vol, probe, pose, 0, 0, 1, p_drop=0.0)
    g = oracle.recon_observe(pts, pose)
    uu = (pts - pose.reshape(3, 4)[:, 3]) @ R     # rows: R^T (p - t)
    assert np.allclose(uu[:, 1], 0.0, atol=1e-9)

    def cells(v):   # cells a coordinate may fall in (both neighbours on a boundary)
        return sorted({int(np.floor(v - 1e-9)), int(np.floor(v + 1e-9))})
    for ux, uy, uz in uu:
        assert any(g[h, w, e] for h in cells(uz / 3) for w in cells((ux + 60) / 3) for e in cells((uy + 60) / 3))
    assert g[:, :, :19].sum() == 0 and g[:, :, 21:].sum() == 0
