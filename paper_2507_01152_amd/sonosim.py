"""Thin ctypes binding of libsonosim.so (C ABI: include/sonosim.h).

Functions carry the C names and only marshal arguments: torch tensors give
device pointers and the HIP stream, numpy/Python sequences give host arrays.
Every step of the simulation runs in the library's HIP kernels; if the
library is not built, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libsonosim.so")

SG_OK, SG_EINVAL, SG_ENOMEM, SG_EHIP, SG_ESTATE, SG_ERANGE = 0, -1, -2, -3, -4, -5
SG_MAX_IMAGE = 1024

# every symbol include/sonosim.h declares
SYMBOLS = (
    "sg_last_error", "sg_version", "sg_create", "sg_destroy", "sg_set_stream", "sg_synchronize",
    "sg_volume_register", "sg_volume_release", "sg_noise_quantiles", "sg_tissue_table_set", "sg_simulate",
    "sg_simulate_noalloc",
    "sg_batch_plan_create", "sg_batch_poses", "sg_batch_set_poses", "sg_batch_step",
    "sg_batch_step_profiled", "sg_batch_status", "sg_autotune",
    "sg_batch_config", "sg_batch_set_config", "sg_batch_plan_destroy",
    "sg_recon_create", "sg_recon_update", "sg_recon_observe", "sg_recon_counts", "sg_recon_points",
    "sg_recon_reset", "sg_recon_destroy",
    "sg_conv_forward", "sg_conv_backward_data", "sg_conv_backward_weight", "sg_valu_probe", "sg_hbm_probe",
    "sg_surr_create", "sg_surr_create_ct", "sg_surr_set_ct_reference", "sg_surr_destroy", "sg_surr_num_params",
    "sg_surr_train_step", "sg_surr_infer", "sg_surr_infer_bf16", "sg_surr_train_pairs", "sg_surr_gan_losses", "sg_surr_disc_num_params",
    "sg_surr_disc_get_params", "sg_surr_disc_get_grads", "sg_surr_disc_set_params",
    "sg_audit_decide", "sg_surr_save", "sg_surr_load", "sg_surr_get_params", "sg_surr_get_grads",
    "sg_surr_set_params", "sg_surr_get_batch", "sg_surr_tensor", "sg_surr_train_step_async",
    "sg_surr_train_pairs_async", "sg_surr_loss_history", "sg_surr_step_count", "sg_surr_set_graph",
)


class SonosimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class sg_volume_desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("spacing_mm", C.c_double * 3), ("labels", C.c_void_p), ("ct_hu", C.c_void_p),
                ("noise_seed", C.c_uint64), ("noise_scales", C.c_int32)]


class sg_tissue(C.Structure):
    _fields_ = [("Z_mrayl", C.c_float), ("alpha_np_cm_mhz", C.c_float), ("mu0", C.c_float),
                ("sigma0", C.c_float), ("mu1", C.c_float)]


class sg_probe(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("dx_mm", C.c_double), ("dy_mm", C.c_double),
                ("f_mhz", C.c_double), ("E0", C.c_double), ("psf_frac", C.c_double),
                ("dr_db", C.c_double), ("n_elev", C.c_int32), ("elev_mm", C.c_double)]


class sg_conv_desc(C.Structure):
    _fields_ = [("N", C.c_int32), ("H", C.c_int32), ("W", C.c_int32), ("C", C.c_int32), ("Co", C.c_int32),
                ("kernel", C.c_int32), ("stride", C.c_int32), ("pad", C.c_int32), ("upsample", C.c_int32)]


class sg_debug_planes(C.Structure):
    _fields_ = [("label", C.c_void_p), ("voxel", C.c_void_p), ("philox", C.c_void_p),
                ("energy", C.c_void_p), ("intensity", C.c_void_p), ("scatter", C.c_void_p)]


_lib = None


def load():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    L = C.CDLL(LIB_PATH)
    P, I32, VP = C.POINTER, C.c_int32, C.c_void_p
    L.sg_last_error.restype = C.c_char_p
    L.sg_version.restype = I32
    sigs = {
        "sg_create": [P(VP), I32, VP],
        "sg_destroy": [VP],
        "sg_set_stream": [VP, VP],
        "sg_synchronize": [VP],
        "sg_volume_register": [VP, P(sg_volume_desc), P(I32)],
        "sg_volume_release": [VP, I32],
        "sg_noise_quantiles": [VP],
        "sg_tissue_table_set": [VP, VP, I32],
        "sg_simulate": [VP, I32, VP, VP, VP, VP, VP, P(sg_debug_planes)],
        "sg_simulate_noalloc": [VP, I32, VP, VP, VP, VP, VP],
        "sg_batch_plan_create": [VP, I32, VP, VP, VP, P(I32)],
        "sg_batch_poses": [VP, I32, P(VP)],
        "sg_batch_set_poses": [VP, I32, VP],
        "sg_batch_step": [VP, I32, VP],
        "sg_batch_step_profiled": [VP, I32, VP, P(C.c_float), P(C.c_float)],
        "sg_batch_status": [VP, I32, P(I32)],
        "sg_autotune": [VP, I32, C.c_char_p],
        "sg_batch_config": [VP, I32, P(I32), P(I32), P(I32), P(I32)],
        "sg_batch_set_config": [VP, I32, I32, I32, I32],
        "sg_recon_create": [VP, I32, I32, VP, C.c_double, C.c_uint64, P(I32)],
        "sg_recon_update": [VP, I32, I32],
        "sg_recon_observe": [VP, I32, VP],
        "sg_recon_counts": [VP, I32, VP, VP],
        "sg_recon_points": [VP, I32, I32, VP, C.c_int64, P(C.c_int64)],
        "sg_recon_reset": [VP, I32, I32],
        "sg_recon_destroy": [VP, I32],
        "sg_batch_plan_destroy": [VP, I32],
        "sg_conv_forward": [VP, P(sg_conv_desc), VP, VP, VP, I32, VP, VP, VP, VP],
        "sg_conv_backward_data": [VP, P(sg_conv_desc), VP, VP, VP, I32],
        "sg_conv_backward_weight": [VP, P(sg_conv_desc), VP, VP, VP, VP],
        "sg_surr_create": [VP, I32, I32, C.c_uint64, P(I32)],
        "sg_valu_probe": [VP, VP],
        "sg_hbm_probe": [VP, VP, VP, C.c_size_t, P(C.c_double)],
        "sg_surr_create_ct": [VP, I32, I32, C.c_uint64, C.c_float, P(I32)],
        "sg_surr_set_ct_reference": [VP, I32, I32, VP, VP, VP, VP],
        "sg_surr_destroy": [VP, I32],
        "sg_surr_train_pairs": [VP, I32, I32, I32, I32, VP, VP, C.c_float, P(C.c_float)],
        "sg_surr_train_pairs_async": [VP, I32, I32, I32, I32, VP, VP, C.c_float],
        "sg_surr_train_step_async": [VP, I32, I32, VP, VP, VP, C.c_float],
        "sg_surr_loss_history": [VP, I32, C.c_int64, I32, VP],
        "sg_surr_step_count": [VP, I32, P(C.c_int64)],
        "sg_surr_set_graph": [VP, I32, I32],
        "sg_surr_gan_losses": [VP, I32, P(C.c_float), P(C.c_float)],
        "sg_surr_disc_num_params": [VP, I32, P(C.c_int64)],
        "sg_surr_disc_get_params": [VP, I32, VP],
        "sg_surr_disc_get_grads": [VP, I32, VP],
        "sg_surr_disc_set_params": [VP, I32, VP],
        "sg_surr_num_params": [VP, I32, P(C.c_int64)],
        "sg_surr_train_step": [VP, I32, I32, VP, VP, VP, C.c_float, P(C.c_float)],
        "sg_surr_infer": [VP, I32, I32, VP, VP, VP, VP, VP, I32, C.c_float, C.c_float, VP, P(I32)],
        "sg_surr_infer_bf16": [VP, I32, I32, VP, VP, VP, VP, VP, I32, C.c_float, C.c_float, VP, P(I32)],
        "sg_audit_decide": [I32, VP, C.c_float, C.c_float, VP, P(I32)],
        "sg_surr_save": [VP, I32, C.c_char_p],
        "sg_surr_load": [VP, I32, C.c_char_p],
        "sg_surr_get_params": [VP, I32, VP],
        "sg_surr_get_grads": [VP, I32, VP],
        "sg_surr_set_params": [VP, I32, VP],
        "sg_surr_get_batch": [VP, I32, VP, VP],
        "sg_surr_tensor": [VP, I32, I32, I32, VP, P(C.c_int64)],
    }
    for name, args in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = I32
    _lib = L
    return L


def _check(status: int, name: str):
    if status != SG_OK:
        msg = load().sg_last_error().decode(errors="replace")
        raise SonosimError(status, f"{name}: {msg}")


def _stream_of(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _dptr(t):
    """Device pointer of a CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _out(t, what: str, elem_size: int, need: int, float32: bool = False):
    """Device pointer of an output tensor the library writes `need` elements
    of `elem_size` bytes into; refuses tensors that are too small, of the
    wrong element size (or not float32 where float32 is written)."""
    if t is None:
        raise ValueError(f"{what}: output tensor is None")
    if t.element_size() != elem_size or (float32 and not t.is_floating_point()):
        raise ValueError(f"{what}: expected {'float32' if float32 else f'{elem_size}-byte'} elements, got {t.dtype}")
    if t.numel() < need:
        raise ValueError(f"{what}: {t.numel()} elements, the call writes {need}")
    return _dptr(t)


def _frames_extent(probes, offs) -> int:
    """Elements of a packed output the frames of `probes` at offsets `offs`
    reach: max(offset + planes * W * H)."""
    if len(probes) == 0:
        return 0
    return int(max(int(o) + max(1, int(getattr(p, "n_elev", 1))) * int(p.W) * int(p.H)
                   for o, p in zip(offs, probes)))


_PLAN_EXTENT = {}   # (context address, plan id) -> output elements a step writes


# ---------------------------------------------------------------------------

def sg_version() -> int:
    return int(load().sg_version())


def sg_create(device: int = 0, stream=None):
    ctx = C.c_void_p()
    _check(load().sg_create(C.byref(ctx), int(device), _stream_of(stream)), "sg_create")
    return ctx


def sg_destroy(ctx):
    _check(load().sg_destroy(ctx), "sg_destroy")
    for k in [k for k in _PLAN_EXTENT if k[0] == ctx.value]:
        del _PLAN_EXTENT[k]


def sg_set_stream(ctx, stream=None):
    _check(load().sg_set_stream(ctx, _stream_of(stream)), "sg_set_stream")


def sg_synchronize(ctx):
    _check(load().sg_synchronize(ctx), "sg_synchronize")


def sg_volume_register(ctx, labels, spacing=(1.0, 1.0, 1.0), ct=None, seed: int = 0, noise_scales: int = 1) -> int:
    """labels: device uint8 tensor [nz, ny, nx]; ct: device int16 tensor or None."""
    nz, ny, nx = labels.shape
    if ct is not None and tuple(ct.shape) != tuple(labels.shape):
        raise ValueError("ct must have the label volume's shape")
    d = sg_volume_desc(nx, ny, nz, (C.c_double * 3)(*[float(s) for s in spacing]), _dptr(labels),
                       _dptr(ct), int(seed) & ((1 << 64) - 1), int(noise_scales))
    vid = C.c_int32()
    _check(load().sg_volume_register(ctx, C.byref(d), C.byref(vid)), "sg_volume_register")
    return int(vid.value)


def sg_volume_release(ctx, vol_id: int):
    _check(load().sg_volume_release(ctx, int(vol_id)), "sg_volume_release")


def sg_noise_quantiles() -> np.ndarray:
    """The quantised standard normal of the multi-scale gate (4096 int32 in
    units of 2^-20, host)."""
    out = np.zeros(4096, dtype=np.int32)
    _check(load().sg_noise_quantiles(out.ctypes.data), "sg_noise_quantiles")
    return out


def sg_tissue_table_set(ctx, table):
    """table: array-like [n_labels, 5] = (Z, alpha, mu0, sigma0, mu1)."""
    t = np.ascontiguousarray(np.asarray(table, dtype=np.float32).reshape(-1, 5))
    _check(load().sg_tissue_table_set(ctx, t.ctypes.data, t.shape[0]), "sg_tissue_table_set")


def probes_array(probes):
    """Host array of sg_probe from objects with W, H, dx, dy, f, E0, psf, dr.
    An sg_probe array (what this returns) passes through unchanged, so a
    caller that serves the same probes every step marshals them once."""
    if _is_probe_array(probes):
        return probes
    arr = (sg_probe * len(probes))()
    for i, p in enumerate(probes):
        arr[i] = p if isinstance(p, sg_probe) else sg_probe(
            int(p.W), int(p.H), float(p.dx), float(p.dy), float(p.f), float(p.E0), float(p.psf), float(p.dr),
            int(getattr(p, "n_elev", 1)), float(getattr(p, "elev", 0.0)))
    return arr


def _is_probe_array(probes):
    return isinstance(probes, C.Array) and probes._type_ is sg_probe


def _pixels(probes):
    """Sum of W * H over the probes (one plane each)."""
    if _is_probe_array(probes):
        dt = np.dtype({"names": ["W", "H"], "formats": [np.int32, np.int32],
                       "offsets": [sg_probe.W.offset, sg_probe.H.offset], "itemsize": C.sizeof(sg_probe)})
        a = np.frombuffer((C.c_char * C.sizeof(probes)).from_buffer(probes), dtype=dt)
        return int((a["W"].astype(np.int64) * a["H"]).sum())
    return sum(int(p.W) * int(p.H) for p in probes)


def sg_simulate(ctx, vol_ids, probes, poses, out, out_offsets, debug: dict | None = None):
    """out: device float32 tensor; debug: dict of device tensors keyed by
    label / voxel / philox / energy / intensity."""
    n = len(probes)
    vids = np.ascontiguousarray(vol_ids, dtype=np.int32)
    pa = probes_array(probes)
    ps = np.ascontiguousarray(poses, dtype=np.float64).reshape(n, 12)
    offs = np.ascontiguousarray(out_offsets, dtype=np.int64)
    if len(vids) != n or len(offs) != n:
        raise ValueError("vol_ids, probes and out_offsets must have one entry per env")
    if (offs < 0).any():
        raise ValueError("out_offsets must be >= 0")
    need = _frames_extent(probes, offs)
    dbg = None
    if debug:
        spec = {"label": (1, 1, False), "voxel": (4, 1, False), "philox": (4, 4, False), "energy": (4, 1, True),
                "intensity": (4, 1, True), "scatter": (4, 1, True)}
        ptrs = []
        for k in ("label", "voxel", "philox", "energy", "intensity", "scatter"):
            t = debug.get(k)
            size, per, f32 = spec[k]
            ptrs.append(None if t is None else _out(t, f"sg_simulate debug {k}", size, per * need, f32))
        dbg = sg_debug_planes(*ptrs)
    _check(load().sg_simulate(ctx, n, vids.ctypes.data, C.cast(pa, C.c_void_p), ps.ctypes.data,
                              _out(out, "sg_simulate", 4, need, True), offs.ctypes.data,
                              C.byref(dbg) if dbg is not None else None), "sg_simulate")


def sg_simulate_noalloc(ctx, vol_ids, probes, poses, out, out_offsets):
    """sg_simulate without allocation (no debug planes); out: device float32 tensor."""
    n = len(probes)
    vids = np.ascontiguousarray(vol_ids, dtype=np.int32)
    pa = probes_array(probes)
    ps = np.ascontiguousarray(poses, dtype=np.float64).reshape(n, 12)
    offs = np.ascontiguousarray(out_offsets, dtype=np.int64)
    if len(vids) != n or len(offs) != n:
        raise ValueError("vol_ids, probes and out_offsets must have one entry per env")
    if (offs < 0).any():
        raise ValueError("out_offsets must be >= 0")
    _check(load().sg_simulate_noalloc(ctx, n, vids.ctypes.data, C.cast(pa, C.c_void_p), ps.ctypes.data,
                                      _out(out, "sg_simulate_noalloc", 4, _frames_extent(probes, offs), True),
                                      offs.ctypes.data), "sg_simulate_noalloc")


def sg_batch_plan_create(ctx, vol_ids, probes, out_offsets) -> int:
    n = len(probes)
    vids = np.ascontiguousarray(vol_ids, dtype=np.int32)
    offs = np.ascontiguousarray(out_offsets, dtype=np.int64)
    pa = probes_array(probes)
    pid = C.c_int32()
    if len(vids) != n or len(offs) != n:
        raise ValueError("vol_ids, probes and out_offsets must have one entry per env")
    _check(load().sg_batch_plan_create(ctx, n, vids.ctypes.data, C.cast(pa, C.c_void_p), offs.ctypes.data,
                                       C.byref(pid)), "sg_batch_plan_create")
    _PLAN_EXTENT[(ctx.value, int(pid.value))] = _frames_extent(probes, offs)
    return int(pid.value)


def _plan_out(ctx, plan_id: int, out, what: str):
    need = _PLAN_EXTENT.get((ctx.value, int(plan_id)))
    if need is None:
        return _dptr(out)   # unknown plan: the library reports it
    return _out(out, what, 4, need, True)


def sg_batch_poses(ctx, plan_id: int) -> int:
    """Device address of the plan's pose buffer (n_envs * 12 float64)."""
    p = C.c_void_p()
    _check(load().sg_batch_poses(ctx, int(plan_id), C.byref(p)), "sg_batch_poses")
    return int(p.value)


def sg_batch_set_poses(ctx, plan_id: int, poses):
    """Upload host poses (n_envs x 12 float64) into the plan's buffer."""
    ps = np.ascontiguousarray(poses, dtype=np.float64)
    _check(load().sg_batch_set_poses(ctx, int(plan_id), ps.ctypes.data), "sg_batch_set_poses")


def sg_batch_step_profiled(ctx, plan_id: int, out):
    """One eager step; returns (ray kernel ms, PSF kernel ms)."""
    a, b = C.c_float(), C.c_float()
    _check(load().sg_batch_step_profiled(ctx, int(plan_id), _plan_out(ctx, plan_id, out, "sg_batch_step_profiled"),
                                         C.byref(a), C.byref(b)), "sg_batch_step_profiled")
    return float(a.value), float(b.value)


def sg_batch_step(ctx, plan_id: int, out):
    _check(load().sg_batch_step(ctx, int(plan_id), _plan_out(ctx, plan_id, out, "sg_batch_step")), "sg_batch_step")


def sg_batch_status(ctx, plan_id: int) -> int:
    n = C.c_int32()
    _check(load().sg_batch_status(ctx, int(plan_id), C.byref(n)), "sg_batch_status")
    return int(n.value)


def sg_autotune(ctx, plan_id: int, cache_path: str | None = None):
    _check(load().sg_autotune(ctx, int(plan_id), None if cache_path is None else cache_path.encode()),
           "sg_autotune")


def sg_batch_config(ctx, plan_id: int):
    """(scanlines_per_item, tile_x, tile_y, chunks) of a plan."""
    a, b, c, d = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(load().sg_batch_config(ctx, int(plan_id), C.byref(a), C.byref(b), C.byref(c), C.byref(d)),
           "sg_batch_config")
    return int(a.value), int(b.value), int(c.value), int(d.value)


def sg_batch_set_config(ctx, plan_id: int, scanlines_per_item: int, tile_x: int, chunks: int = 1):
    _check(load().sg_batch_set_config(ctx, int(plan_id), int(scanlines_per_item), int(tile_x), int(chunks)),
           "sg_batch_set_config")


def sg_batch_plan_destroy(ctx, plan_id: int):
    _check(load().sg_batch_plan_destroy(ctx, int(plan_id)), "sg_batch_plan_destroy")
    _PLAN_EXTENT.pop((ctx.value, int(plan_id)), None)


# ---------------------------------------------------------------------------
# convolution ops and the surrogate

def conv_desc(N, H, W, C_, Co, kernel=3, stride=1, pad=1, upsample=0):
    return sg_conv_desc(N, H, W, C_, Co, kernel, stride, pad, upsample)


def sg_conv_forward(ctx, desc, x, w, bias=None, relu=False, skip=None, y=None, y_skip=None, y_f32=None):
    """x, w, skip, y, y_skip: device bf16 tensors (torch.int16/uint16 storage or bfloat16);
    bias, y_f32: device float32."""
    _check(load().sg_conv_forward(ctx, C.byref(desc), _dptr(x), _dptr(w), _dptr(bias), int(bool(relu)), _dptr(skip),
                                  _dptr(y), _dptr(y_skip), _dptr(y_f32)), "sg_conv_forward")


def sg_conv_backward_data(ctx, desc, dy, w, dx, accumulate=False):
    _check(load().sg_conv_backward_data(ctx, C.byref(desc), _dptr(dy), _dptr(w), _dptr(dx), int(bool(accumulate))),
           "sg_conv_backward_data")


def sg_conv_backward_weight(ctx, desc, x, dy, dw, db=None):
    _check(load().sg_conv_backward_weight(ctx, C.byref(desc), _dptr(x), _dptr(dy), _dptr(dw), _dptr(db)),
           "sg_conv_backward_weight")


def sg_surr_create(ctx, H=256, W=128, seed=0) -> int:
    sid = C.c_int32()
    _check(load().sg_surr_create(ctx, int(H), int(W), int(seed) & ((1 << 64) - 1), C.byref(sid)), "sg_surr_create")
    return int(sid.value)


def sg_surr_create_ct(ctx, H=256, W=128, seed=0, adv_weight=0.0) -> int:
    sid = C.c_int32()
    _check(load().sg_surr_create_ct(ctx, int(H), int(W), int(seed) & ((1 << 64) - 1), float(adv_weight),
                                    C.byref(sid)), "sg_surr_create_ct")
    return int(sid.value)


def sg_surr_set_ct_reference(ctx, sid, vol_ids, probes, poses) -> np.ndarray:
    """Pooled reference histogram (4096 int64 counts) of the given frames."""
    n = len(probes)
    vids = np.ascontiguousarray(vol_ids, dtype=np.int32)
    pa = probes_array(probes)
    ps = np.ascontiguousarray(poses, dtype=np.float64).reshape(n, 12)
    h = np.zeros(4096, dtype=np.int64)
    _check(load().sg_surr_set_ct_reference(ctx, int(sid), n, vids.ctypes.data, C.cast(pa, C.c_void_p),
                                           ps.ctypes.data, h.ctypes.data), "sg_surr_set_ct_reference")
    return h


def _pairs_shape(inp, target):
    if target.dim() != 3 or target.element_size() != 4 or inp.element_size() != 2:
        raise ValueError("target must be float32 [n, H, W] and inp 2-byte [n, H, W, 8]")
    n, H, W = (int(v) for v in target.shape)
    if tuple(inp.shape) != (n, H, W, 8):
        raise ValueError(f"inp shape {tuple(inp.shape)} != {(n, H, W, 8)}")
    return n, H, W


def sg_surr_train_pairs(ctx, sid, inp, target, lr) -> float:
    """inp: device bf16 bits (2-byte tensor, n x H x W x 8); target: device float32 (n x H x W)."""
    n, H, W = _pairs_shape(inp, target)
    loss = C.c_float()
    _check(load().sg_surr_train_pairs(ctx, int(sid), n, H, W, _dptr(inp), _dptr(target), float(lr), C.byref(loss)),
           "sg_surr_train_pairs")
    return float(loss.value)


def sg_surr_train_pairs_async(ctx, sid, inp, target, lr) -> None:
    """As sg_surr_train_pairs, enqueued without reading the loss back."""
    n, H, W = _pairs_shape(inp, target)
    _check(load().sg_surr_train_pairs_async(ctx, int(sid), n, H, W, _dptr(inp), _dptr(target), float(lr)),
           "sg_surr_train_pairs_async")


def sg_surr_loss_history(ctx, sid, first_step, count) -> np.ndarray:
    """(count, 3) float32: L1, L_D, L_adv of steps first_step .. first_step + count - 1 (1-based)."""
    out = np.zeros((int(count), 3), dtype=np.float32)
    _check(load().sg_surr_loss_history(ctx, int(sid), int(first_step), int(count), out.ctypes.data),
           "sg_surr_loss_history")
    return out


def sg_surr_step_count(ctx, sid) -> int:
    n = C.c_int64()
    _check(load().sg_surr_step_count(ctx, int(sid), C.byref(n)), "sg_surr_step_count")
    return int(n.value)


def sg_surr_set_graph(ctx, sid, enable: bool) -> None:
    _check(load().sg_surr_set_graph(ctx, int(sid), 1 if enable else 0), "sg_surr_set_graph")


def sg_surr_gan_losses(ctx, sid):
    """(L_D, L_adv) of the last training step."""
    a, b = C.c_float(), C.c_float()
    _check(load().sg_surr_gan_losses(ctx, int(sid), C.byref(a), C.byref(b)), "sg_surr_gan_losses")
    return float(a.value), float(b.value)


def sg_surr_disc_num_params(ctx, sid) -> int:
    n = C.c_int64()
    _check(load().sg_surr_disc_num_params(ctx, int(sid), C.byref(n)), "sg_surr_disc_num_params")
    return int(n.value)


def sg_surr_disc_get_params(ctx, sid) -> np.ndarray:
    h = np.zeros(sg_surr_disc_num_params(ctx, sid), dtype=np.float32)
    _check(load().sg_surr_disc_get_params(ctx, int(sid), h.ctypes.data), "sg_surr_disc_get_params")
    return h


def sg_surr_disc_get_grads(ctx, sid) -> np.ndarray:
    h = np.zeros(sg_surr_disc_num_params(ctx, sid), dtype=np.float32)
    _check(load().sg_surr_disc_get_grads(ctx, int(sid), h.ctypes.data), "sg_surr_disc_get_grads")
    return h


def sg_surr_disc_set_params(ctx, sid, host):
    h = np.ascontiguousarray(host, dtype=np.float32)
    assert h.size == sg_surr_disc_num_params(ctx, sid)
    _check(load().sg_surr_disc_set_params(ctx, int(sid), h.ctypes.data), "sg_surr_disc_set_params")


def sg_surr_destroy(ctx, sid):
    _check(load().sg_surr_destroy(ctx, int(sid)), "sg_surr_destroy")


def sg_surr_num_params(ctx, sid) -> int:
    n = C.c_int64()
    _check(load().sg_surr_num_params(ctx, int(sid), C.byref(n)), "sg_surr_num_params")
    return int(n.value)


def sg_surr_train_step(ctx, sid, vol_ids, probes, poses, lr) -> float:
    n = len(probes)
    vids = np.ascontiguousarray(vol_ids, dtype=np.int32)
    pa = probes_array(probes)
    ps = np.ascontiguousarray(poses, dtype=np.float64).reshape(n, 12)
    loss = C.c_float()
    _check(load().sg_surr_train_step(ctx, int(sid), n, vids.ctypes.data, C.cast(pa, C.c_void_p), ps.ctypes.data,
                                     float(lr), C.byref(loss)), "sg_surr_train_step")
    return float(loss.value)


def sg_surr_train_step_async(ctx, sid, vol_ids, probes, poses, lr) -> None:
    """As sg_surr_train_step, enqueued without reading the loss back."""
    n = len(probes)
    vids = np.ascontiguousarray(vol_ids, dtype=np.int32)
    pa = probes_array(probes)
    ps = np.ascontiguousarray(poses, dtype=np.float64).reshape(n, 12)
    _check(load().sg_surr_train_step_async(ctx, int(sid), n, vids.ctypes.data, C.cast(pa, C.c_void_p),
                                           ps.ctypes.data, float(lr)), "sg_surr_train_step_async")


def sg_surr_infer(ctx, sid, vol_ids, probes, poses, out, audit_envs=(), psnr_min=30.0, max_fail_frac=0.25):
    """Returns (psnr of the audited envs, number of frames rendered by physics)."""
    n = len(probes)
    vids = np.ascontiguousarray(vol_ids, dtype=np.int32)
    pa = probes_array(probes)
    ps = np.ascontiguousarray(poses, dtype=np.float64).reshape(n, 12)
    au = np.ascontiguousarray(audit_envs, dtype=np.int32)
    if len(vids) != n:
        raise ValueError("vol_ids and probes must have one entry per env")
    need = _pixels(probes)
    psnr = np.zeros(max(1, len(au)), dtype=np.float32)
    nf = C.c_int32()
    _check(load().sg_surr_infer(ctx, int(sid), n, vids.ctypes.data, C.cast(pa, C.c_void_p), ps.ctypes.data,
                                _out(out, "sg_surr_infer", 4, need, True),
                                au.ctypes.data if len(au) else None, len(au), float(psnr_min), float(max_fail_frac),
                                psnr.ctypes.data if len(au) else None, C.byref(nf)), "sg_surr_infer")
    return psnr[:len(au)], int(nf.value)


def sg_surr_infer_bf16(ctx, sid, vol_ids, probes, poses, out, audit_envs=(), psnr_min=30.0, max_fail_frac=0.25):
    """sg_surr_infer with bf16 frames: out is a 2-byte device tensor (bfloat16
    or int16 storage) of n x H x W elements."""
    n = len(probes)
    vids = np.ascontiguousarray(vol_ids, dtype=np.int32)
    pa = probes_array(probes)
    ps = np.ascontiguousarray(poses, dtype=np.float64).reshape(n, 12)
    au = np.ascontiguousarray(audit_envs, dtype=np.int32)
    if len(vids) != n:
        raise ValueError("vol_ids and probes must have one entry per env")
    need = _pixels(probes)
    psnr = np.zeros(max(1, len(au)), dtype=np.float32)
    nf = C.c_int32()
    _check(load().sg_surr_infer_bf16(ctx, int(sid), n, vids.ctypes.data, C.cast(pa, C.c_void_p), ps.ctypes.data,
                                     _out(out, "sg_surr_infer_bf16", 2, need), au.ctypes.data if len(au) else None,
                                     len(au), float(psnr_min), float(max_fail_frac),
                                     psnr.ctypes.data if len(au) else None, C.byref(nf)), "sg_surr_infer_bf16")
    return psnr[:len(au)], int(nf.value)


def sg_audit_decide(psnr, psnr_min, max_fail_frac):
    p = np.ascontiguousarray(psnr, dtype=np.float32)
    fb = np.zeros(max(1, len(p)), dtype=np.int32)
    whole = C.c_int32()
    _check(load().sg_audit_decide(len(p), p.ctypes.data if len(p) else None, float(psnr_min), float(max_fail_frac),
                                  fb.ctypes.data, C.byref(whole)), "sg_audit_decide")
    return fb[:len(p)].astype(bool), bool(whole.value)


def sg_surr_save(ctx, sid, path):
    _check(load().sg_surr_save(ctx, int(sid), str(path).encode()), "sg_surr_save")


def sg_surr_load(ctx, sid, path):
    _check(load().sg_surr_load(ctx, int(sid), str(path).encode()), "sg_surr_load")


def sg_surr_get_params(ctx, sid) -> np.ndarray:
    h = np.zeros(sg_surr_num_params(ctx, sid), dtype=np.float32)
    _check(load().sg_surr_get_params(ctx, int(sid), h.ctypes.data), "sg_surr_get_params")
    return h


def sg_surr_get_grads(ctx, sid) -> np.ndarray:
    h = np.zeros(sg_surr_num_params(ctx, sid), dtype=np.float32)
    _check(load().sg_surr_get_grads(ctx, int(sid), h.ctypes.data), "sg_surr_get_grads")
    return h


def sg_surr_set_params(ctx, sid, params):
    h = np.ascontiguousarray(params, dtype=np.float32)
    if h.size != sg_surr_num_params(ctx, sid):
        raise ValueError("wrong parameter count")
    _check(load().sg_surr_set_params(ctx, int(sid), h.ctypes.data), "sg_surr_set_params")


(SURR_T_ACT, SURR_T_GRAD, SURR_T_YHAT, SURR_T_TARGET, SURR_T_GY, SURR_T_MOM1, SURR_T_MOM2, SURR_T_DISC_ACT,
 SURR_T_DISC_GRAD, SURR_T_DISC_LOGITS, SURR_T_DISC_GLOG, SURR_T_DISC_MOM1, SURR_T_DISC_MOM2, SURR_T_DSCAN) = range(14)
SURR_TENSORS = ("X", "T1", "E0", "T2", "E1", "T3", "E2", "T4", "E3", "T5", "B4", "U3", "S3", "D3", "U2", "S2",
                "D2", "U1", "S1", "D1", "U0", "S0", "D0", "A0")


def sg_surr_tensor(ctx, sid, kind: int, index: int = 0) -> np.ndarray:
    """Flat host copy of a tensor of the last training step (uint16 bf16 bits
    for the activation kinds, float32 otherwise)."""
    n = C.c_int64()
    _check(load().sg_surr_tensor(ctx, int(sid), int(kind), int(index), None, C.byref(n)), "sg_surr_tensor")
    bf = kind in (SURR_T_ACT, SURR_T_DISC_ACT, SURR_T_DSCAN)
    h = np.zeros(int(n.value), dtype=np.uint16 if bf else np.float32)
    _check(load().sg_surr_tensor(ctx, int(sid), int(kind), int(index), h.ctypes.data, C.byref(n)), "sg_surr_tensor")
    return h


def sg_surr_get_batch(ctx, sid, n, H, W):
    """(input bf16 bits uint16 [n,H,W,8], target float32 [n,H,W]) of the last training step."""
    x = np.zeros((n, H, W, 8), dtype=np.uint16)
    y = np.zeros((n, H, W), dtype=np.float32)
    _check(load().sg_surr_get_batch(ctx, int(sid), x.ctypes.data, y.ctypes.data), "sg_surr_get_batch")
    return x, y


# ---------------------------------------------------------------------------
# reconstruction observation (bone-surface task)

def sg_recon_create(ctx, plan_id: int, capacity: int, bone_labels=None, p_miss: float = 0.2, seed: int = 0) -> int:
    """bone_labels: iterable of label values (None: label 3)."""
    bone = None
    if bone_labels is not None:
        bone = np.zeros(256, dtype=np.uint8)
        bone[list(bone_labels)] = 1
    rid = C.c_int32()
    _check(load().sg_recon_create(ctx, int(plan_id), int(capacity), None if bone is None else bone.ctypes.data,
                                  float(p_miss), int(seed) & ((1 << 64) - 1), C.byref(rid)), "sg_recon_create")
    return int(rid.value)


def sg_recon_update(ctx, recon_id: int, step: int):
    _check(load().sg_recon_update(ctx, int(recon_id), int(step)), "sg_recon_update")


def sg_recon_observe(ctx, recon_id: int, grids):
    """grids: device uint8 tensor of n_envs * 40^3 elements."""
    _check(load().sg_recon_observe(ctx, int(recon_id), _dptr(grids)), "sg_recon_observe")


def sg_recon_counts(ctx, recon_id: int, n_envs: int):
    stored = np.zeros(n_envs, dtype=np.int64)
    over = np.zeros(n_envs, dtype=np.int64)
    _check(load().sg_recon_counts(ctx, int(recon_id), stored.ctypes.data, over.ctypes.data), "sg_recon_counts")
    return stored, over


def sg_recon_points(ctx, recon_id: int, env: int, max_points: int) -> np.ndarray:
    buf = np.zeros((max(1, max_points), 3), dtype=np.float64)
    n = C.c_int64()
    _check(load().sg_recon_points(ctx, int(recon_id), int(env), buf.ctypes.data, int(max_points), C.byref(n)),
           "sg_recon_points")
    return buf[:n.value].copy()


def sg_recon_reset(ctx, recon_id: int, env: int = -1):
    _check(load().sg_recon_reset(ctx, int(recon_id), int(env)), "sg_recon_reset")


def sg_recon_destroy(ctx, recon_id: int):
    _check(load().sg_recon_destroy(ctx, int(recon_id)), "sg_recon_destroy")


def sg_valu_probe(ctx):
    """Lane-op rates: (FP32 FMA two-operand, xor/add, 32x32->64 mad, FP32 FMA three-operand)."""
    r = np.zeros(4, dtype=np.float64)
    _check(load().sg_valu_probe(ctx, r.ctypes.data), "sg_valu_probe")
    return tuple(float(v) for v in r)


def sg_hbm_probe(ctx, src, dst):
    """Device copy src -> dst (same byte size); returns bytes read + written per second."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("sg_hbm_probe: src and dst sizes differ")
    r = C.c_double()
    _check(load().sg_hbm_probe(ctx, _dptr(src), _dptr(dst), nbytes, C.byref(r)), "sg_hbm_probe")
    return r.value
