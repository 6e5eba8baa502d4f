"""ctypes binding of libdtsdf.so (the C ABI declared in include/dtsdf.h).

Argument marshalling only: device buffers are torch tensors on the HIP device, passed by
pointer together with torch's current stream; every step of the computation runs in the
library's HIP kernels.  There is no fallback: if the library is missing, importing this module
raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdtsdf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c \"import "
                      "__graft_entry__ as g; g.build()\"` (hipcc, gfx950)")
_lib = ctypes.CDLL(LIB_PATH)

OK, E_INVAL, E_NOMEM, E_CAPACITY, E_HIP, E_DEGENERATE, E_BUSY = range(7)
SDF_F32, SDF_F16, SDF_I16 = 0, 1, 2
RENDER_ALONE = 1
W_F32, W_U8 = 0, 1
ICP_W_CONST, ICP_W_DEPTH = 0, 1


class DtsdfError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {_lib.dtsdf_status_string(status).decode()} ({status})")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("voxel_size", ctypes.c_float), ("truncation", ctypes.c_float),
                ("theta", ctypes.c_float), ("w_carve", ctypes.c_float),
                ("w_max", ctypes.c_float), ("w_min", ctypes.c_float),
                ("lattice_step", ctypes.c_float), ("sdf_fmt", ctypes.c_int32),
                ("w_fmt", ctypes.c_int32), ("with_color", ctypes.c_int32),
                ("brick_capacity", ctypes.c_uint32), ("hash_buckets", ctypes.c_uint32),
                ("dense", ctypes.c_int32), ("dense_lo", ctypes.c_int32 * 3),
                ("dense_hi", ctypes.c_int32 * 3)]


class _Info(ctypes.Structure):
    _fields_ = [("bricks", ctypes.c_int64), ("capacity", ctypes.c_int64),
                ("blocks", ctypes.c_int64), ("hash_buckets", ctypes.c_int64),
                ("dropped", ctypes.c_int64), ("device_bytes", ctypes.c_int64)]


class _Intr(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


class _RenderOut(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("vertex", ctypes.c_void_p),
                ("normal", ctypes.c_void_p), ("rgba", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("trace_bricks", ctypes.c_void_p),
                ("trace_color", ctypes.c_void_p), ("trace_slots", ctypes.c_void_p),
                ("trace_counts", ctypes.c_void_p), ("flags", ctypes.c_int32)]


class _Blob(ctypes.Structure):
    _fields_ = [("n_bricks", ctypes.c_int64), ("keys", ctypes.c_void_p), ("sdf", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("rgb", ctypes.c_void_p), ("wc", ctypes.c_void_p)]


class _Stats(ctypes.Structure):
    _fields_ = [("new_bricks", ctypes.c_int64), ("dropped", ctypes.c_int64),
                ("bricks", ctypes.c_int64), ("visited_bricks", ctypes.c_int64),
                ("updated_voxels", ctypes.c_int64), ("color_voxels", ctypes.c_int64)]


class _Image(ctypes.Structure):
    _fields_ = [("vertex", ctypes.c_void_p), ("normal", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("intr", _Intr)]


class _IcpParams(ctypes.Structure):
    _fields_ = [("max_dist", ctypes.c_float), ("max_angle_deg", ctypes.c_float),
                ("weight", ctypes.c_int32), ("z_min", ctypes.c_float),
                ("min_inliers_per_dim", ctypes.c_int32), ("compensated", ctypes.c_int32)]


class _IcpResult(ctypes.Structure):
    _fields_ = [("xi", ctypes.c_double * 7), ("H", ctypes.c_double * 49),
                ("g", ctypes.c_double * 7), ("error", ctypes.c_double),
                ("inliers", ctypes.c_int64), ("step_norm", ctypes.c_double),
                ("status", ctypes.c_int32), ("photometric", ctypes.c_int32)]


class _Photo(ctypes.Structure):
    _fields_ = [("live_intensity", ctypes.c_void_p), ("ref_intensity", ctypes.c_void_p),
                ("ref_intr", _Intr), ("T_ref_model", ctypes.c_double * 16),
                ("lambda_", ctypes.c_float), ("max_error", ctypes.c_float)]


class _RenderReq(ctypes.Structure):
    _fields_ = [("intr", _Intr), ("T_world_cam", ctypes.c_double * 16),
                ("z_near", ctypes.c_float), ("z_far", ctypes.c_float), ("out", _RenderOut)]


class _IcpReq(ctypes.Structure):
    _fields_ = [("live", _Image), ("model", _Image), ("dim", ctypes.c_int32),
                ("params", _IcpParams), ("pose", ctypes.c_void_p), ("active", ctypes.c_void_p),
                ("min_step", ctypes.c_double), ("result", ctypes.c_void_p),
                ("photo", ctypes.c_void_p)]


class _LmState(ctypes.Structure):
    _fields_ = [("T", ctypes.c_double * 16), ("T_acc", ctypes.c_double * 16),
                ("H", ctypes.c_double * 49), ("g", ctypes.c_double * 7), ("F", ctypes.c_double),
                ("h", ctypes.c_double * 7), ("mu", ctypes.c_double), ("nu", ctypes.c_double),
                ("tau", ctypes.c_double), ("started", ctypes.c_int32),
                ("accepted", ctypes.c_int32)]


class _DepthFilterParams(ctypes.Structure):
    _fields_ = [("support_rel", ctypes.c_float), ("min_support", ctypes.c_int32),
                ("sigma_d", ctypes.c_float), ("sigma_r", ctypes.c_float),
                ("radius", ctypes.c_int32)]


ICP_RESULT_BYTES = ctypes.sizeof(_IcpResult)


_V = ctypes.c_void_p
_D16 = ctypes.POINTER(ctypes.c_double)

class _RecombineState(ctypes.Structure):
    _fields_ = [("boot_frames", ctypes.c_int32), ("stale_frames", ctypes.c_int32),
                ("max_translation", ctypes.c_double), ("max_angle", ctypes.c_double),
                ("frames", ctypes.c_int64), ("since", ctypes.c_int64),
                ("last_pose", ctypes.c_double * 16), ("has_pose", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


EXPORTED = ["dtsdf_create", "dtsdf_destroy", "dtsdf_get_info", "dtsdf_integrate",
            "dtsdf_render", "dtsdf_render_batch", "dtsdf_export", "dtsdf_import",
            "dtsdf_vertex_normal", "dtsdf_depth_downsample", "icp_step", "icp_step_batch",
            "dtsdf_volume_create", "dtsdf_combine", "dtsdf_recombine_decide",
            "icp_step_rgb", "icp_step_lm", "dtsdf_intensity", "dtsdf_intensity_downsample",
            "dtsdf_depth_filter", "dtsdf_normal_filter", "dtsdf_depth_error", "dtsdf_recycle",
            "dtsdf_integrate_normals", "icp_step_batch_iters",
            "icp_step_batch_iters_noalloc", "dtsdf_level_intrinsics", "dtsdf_icp_pyramid",
            "dtsdf_status_string"]

_lib.dtsdf_status_string.restype = ctypes.c_char_p
_lib.dtsdf_status_string.argtypes = [ctypes.c_int]
_lib.dtsdf_create.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_V)]
_lib.dtsdf_destroy.argtypes = [_V]
_lib.dtsdf_get_info.argtypes = [_V, ctypes.POINTER(_Info)]
_lib.dtsdf_integrate.argtypes = [_V, _V, _V, ctypes.POINTER(_Intr), _D16, ctypes.c_float, _V,
                                 ctypes.POINTER(_Stats)]
_lib.dtsdf_render.argtypes = [_V, ctypes.POINTER(_Intr), _D16, ctypes.c_float, ctypes.c_float,
                              ctypes.POINTER(_RenderOut), _V]
_lib.dtsdf_export.argtypes = [_V, ctypes.POINTER(_Blob)]
_lib.dtsdf_import.argtypes = [_V, ctypes.POINTER(_Blob)]
_lib.dtsdf_vertex_normal.argtypes = [_V, ctypes.POINTER(_Intr), ctypes.c_float, _V, _V, _V]
_lib.dtsdf_depth_downsample.argtypes = [_V, ctypes.c_int32, ctypes.c_int32, _V, _V]
_lib.icp_step.argtypes = [ctypes.POINTER(_Image), ctypes.POINTER(_Image), ctypes.c_int32,
                          ctypes.POINTER(_IcpParams), _D16, ctypes.POINTER(_IcpResult), _V]
_lib.dtsdf_render_batch.argtypes = [_V, ctypes.c_int32, ctypes.POINTER(_RenderReq), _V]
_lib.icp_step_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(_IcpReq), _V]
_lib.icp_step_batch_iters.argtypes = [ctypes.c_int32, ctypes.POINTER(_IcpReq), ctypes.c_int32, _V]
_lib.dtsdf_icp_pyramid.argtypes = [ctypes.c_int32, ctypes.POINTER(_IcpReq),
                                   ctypes.POINTER(ctypes.c_int32), _V]
_lib.icp_step_batch_iters_noalloc.argtypes = [ctypes.c_int32, ctypes.POINTER(_IcpReq),
                                              ctypes.c_int32, _V]
NOALLOC_MAX_REQUESTS = 16
_lib.icp_step_rgb.argtypes = [ctypes.POINTER(_Image), ctypes.POINTER(_Image),
                              ctypes.POINTER(_Photo), ctypes.c_int32,
                              ctypes.POINTER(_IcpParams), _D16, ctypes.POINTER(_IcpResult), _V]
_lib.icp_step_lm.argtypes = [ctypes.POINTER(_Image), ctypes.POINTER(_Image),
                             ctypes.POINTER(_Photo), ctypes.c_int32, ctypes.POINTER(_IcpParams),
                             ctypes.POINTER(_LmState), ctypes.POINTER(_IcpResult), _V]
_lib.dtsdf_integrate_normals.argtypes = [_V, _V, _V, _V, ctypes.POINTER(_Intr), _D16,
                                         ctypes.c_float, _V, ctypes.POINTER(_Stats)]
_lib.dtsdf_recycle.argtypes = [_V, ctypes.c_float, ctypes.POINTER(ctypes.c_int64), _V]
_lib.dtsdf_depth_filter.argtypes = [_V, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(_DepthFilterParams), _V, _V]
_lib.dtsdf_normal_filter.argtypes = [_V, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_int32, _V, _V]
_lib.dtsdf_depth_error.argtypes = [_V, _V, ctypes.c_int32, ctypes.c_int32, _V, _V]
_lib.dtsdf_intensity.argtypes = [_V, ctypes.c_int32, ctypes.c_int32, _V, _V]
_lib.dtsdf_intensity_downsample.argtypes = [_V, ctypes.c_int32, ctypes.c_int32, _V, _V]
_lib.dtsdf_volume_create.argtypes = [_V, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(_V)]
_lib.dtsdf_combine.argtypes = [_V, _V, _D16, _D16, ctypes.POINTER(_Intr), ctypes.c_float,
                               ctypes.c_int32, _V]
_lib.dtsdf_recombine_decide.argtypes = [ctypes.POINTER(_RecombineState), _D16,
                                        ctypes.POINTER(ctypes.c_int32)]
_lib.dtsdf_level_intrinsics.argtypes = [ctypes.POINTER(_Intr), ctypes.c_int32,
                                        ctypes.POINTER(_Intr)]
for _f in EXPORTED:
    if _f != "dtsdf_status_string":
        getattr(_lib, _f).restype = ctypes.c_int


def _check(status: int, what: str, allow=()):
    if status != OK and status not in allow:
        raise DtsdfError(status, what)
    return status


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t: Optional[torch.Tensor], dtype, numel=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device buffers must be HIP tensors")
    if t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("device buffers must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _intr(cam) -> _Intr:
    return _Intr(int(cam.width), int(cam.height), float(cam.fx), float(cam.fy), float(cam.cx),
                 float(cam.cy))


def _pose(T) -> ctypes.Array:
    a = np.ascontiguousarray(np.asarray(T, np.float64).reshape(16))
    return (ctypes.c_double * 16)(*a.tolist())


@dataclasses.dataclass
class Params:
    voxel_size: float
    truncation: float
    theta: float = math.pi / 3.0
    w_carve: float = 0.1
    w_max: float = 63.75
    w_min: float = 1e-4
    lattice_step: Optional[float] = None
    sdf_fmt: int = SDF_F32
    w_fmt: int = W_F32
    with_color: bool = True
    brick_capacity: int = 1 << 16
    hash_buckets: int = 1 << 17
    dense_lo: Optional[Sequence[int]] = None
    dense_hi: Optional[Sequence[int]] = None

    def c_struct(self) -> _Params:
        p = _Params()
        p.voxel_size = self.voxel_size
        p.truncation = self.truncation
        p.theta = self.theta
        p.w_carve = self.w_carve
        p.w_max = self.w_max
        p.w_min = self.w_min
        p.lattice_step = self.lattice_step if self.lattice_step is not None else 0.5 * self.voxel_size
        p.sdf_fmt = self.sdf_fmt
        p.w_fmt = self.w_fmt
        p.with_color = int(self.with_color)
        p.brick_capacity = self.brick_capacity
        p.hash_buckets = self.hash_buckets
        p.dense = 1 if self.dense_lo is not None else 0
        for k in range(3):
            p.dense_lo[k] = int(self.dense_lo[k]) if self.dense_lo is not None else 0
            p.dense_hi[k] = int(self.dense_hi[k]) if self.dense_hi is not None else 0
        return p


class Map:
    """A Directional TSDF resident in device memory."""

    def __init__(self, params: Params):
        self.params = params
        h = _V()
        _check(_lib.dtsdf_create(ctypes.byref(params.c_struct()), ctypes.byref(h)), "dtsdf_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.dtsdf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        i = _Info()
        _check(_lib.dtsdf_get_info(self._h, ctypes.byref(i)), "dtsdf_get_info")
        return {k: getattr(i, k) for k, _ in _Info._fields_}

    def integrate(self, depth: torch.Tensor, rgb: Optional[torch.Tensor], cam, T_wc,
                  depth_scale: float = 1.0, stats: bool = False, stream=None,
                  normal: Optional[torch.Tensor] = None):
        """Fuse one frame; ``normal`` (planar (3, H, W) camera-frame unit normals, e.g. from
        normal_filter) replaces the cross-product normals of the depth."""
        H, W = int(cam.height), int(cam.width)
        st = _Stats() if stats else None
        dp = _dev_ptr(depth, torch.float32, H * W)
        cp = _dev_ptr(rgb, torch.uint8, H * W * 3) if rgb is not None else None
        sp = ctypes.byref(st) if st is not None else None
        if normal is None:
            status = _lib.dtsdf_integrate(self._h, dp, cp, ctypes.byref(_intr(cam)), _pose(T_wc),
                                          depth_scale, _stream(stream), sp)
        else:
            status = _lib.dtsdf_integrate_normals(
                self._h, dp, _dev_ptr(normal, torch.float32, 3 * H * W), cp,
                ctypes.byref(_intr(cam)), _pose(T_wc), depth_scale, _stream(stream), sp)
        _check(status, "dtsdf_integrate", allow=(E_CAPACITY,))
        if stats:
            return dict(status=status, new_bricks=st.new_bricks, dropped=st.dropped,
                        bricks=st.bricks, visited_bricks=st.visited_bricks,
                        updated_voxels=st.updated_voxels, color_voxels=st.color_voxels)
        return status

    def _render_out(self, cam, out: dict) -> _RenderOut:
        H, W = int(cam.height), int(cam.width)
        cap, nb = self.params.brick_capacity, self.params.hash_buckets
        return _RenderOut(_dev_ptr(out.get("depth"), torch.float32, H * W),
                          _dev_ptr(out.get("vertex"), torch.float32, 3 * H * W),
                          _dev_ptr(out.get("normal"), torch.float32, 3 * H * W),
                          _dev_ptr(out.get("rgba"), torch.uint8, 4 * H * W),
                          _dev_ptr(out.get("mask"), torch.uint8, H * W),
                          _dev_ptr(out.get("trace_bricks"), torch.uint8, cap),
                          _dev_ptr(out.get("trace_color"), torch.uint8, cap),
                          _dev_ptr(out.get("trace_slots"), torch.uint8, nb),
                          _dev_ptr(out.get("trace_counts"), torch.int32, 4 * H * W),
                          RENDER_ALONE if out.get("alone", False) else 0)

    def render_batch(self, views, stream=None) -> None:
        """views: list of (cam, T_wc, z_near, z_far, out dict of preallocated tensors)."""
        n = len(views)
        reqs = (_RenderReq * n)()
        for i, (cam, T, zn, zf, out) in enumerate(views):
            reqs[i].intr = _intr(cam)
            reqs[i].T_world_cam = _pose(T)
            reqs[i].z_near = zn
            reqs[i].z_far = zf
            reqs[i].out = self._render_out(cam, out)
        _check(_lib.dtsdf_render_batch(self._h, n, reqs, _stream(stream)), "dtsdf_render_batch")

    def render(self, cam, T_wc, z_near: float = 0.2, z_far: float = 10.0,
               out: Optional[dict] = None, outputs=("depth", "vertex", "normal", "rgba", "mask"),
               stream=None, alone: bool = False) -> dict:
        """Renders a view into `out` (preallocated tensors) or new tensors of `outputs`;
        alone: every ray marches alone (DTSDF_RENDER_ALONE)."""
        H, W = int(cam.height), int(cam.width)
        dev = torch.device("cuda", torch.cuda.current_device())
        if out is None:
            out = {}
            shapes = dict(depth=((H, W), torch.float32), vertex=((3, H, W), torch.float32),
                          normal=((3, H, W), torch.float32), rgba=((H, W, 4), torch.uint8),
                          mask=((H, W), torch.uint8))
            for k in outputs:
                shp, dt = shapes[k]
                out[k] = torch.empty(shp, dtype=dt, device=dev)
        ro = self._render_out(cam, dict(out, alone=alone))
        _check(_lib.dtsdf_render(self._h, ctypes.byref(_intr(cam)), _pose(T_wc), z_near, z_far,
                                 ctypes.byref(ro), _stream(stream)), "dtsdf_render")
        return out

    def recycle(self, t_free: float = 0.9, stream=None) -> int:
        """Return bricks without surface to the pool (see dtsdf_recycle); returns how many."""
        n = ctypes.c_int64(0)
        _check(_lib.dtsdf_recycle(self._h, t_free, ctypes.byref(n), _stream(stream)),
               "dtsdf_recycle")
        return int(n.value)

    def export(self) -> dict:
        b = _Blob()
        _check(_lib.dtsdf_export(self._h, ctypes.byref(b)), "dtsdf_export")
        n = b.n_bricks
        out = dict(keys=np.zeros((n, 4), np.int32), sdf=np.zeros((n, 512), np.float32),
                   w=np.zeros((n, 512), np.float32), rgb=np.zeros((n, 512, 3), np.uint8),
                   wc=np.zeros((n, 512), np.float32))
        b.keys = out["keys"].ctypes.data
        b.sdf = out["sdf"].ctypes.data
        b.w = out["w"].ctypes.data
        b.rgb = out["rgb"].ctypes.data
        b.wc = out["wc"].ctypes.data
        _check(_lib.dtsdf_export(self._h, ctypes.byref(b)), "dtsdf_export")
        return out

    def load(self, blob: dict) -> None:
        keys = np.ascontiguousarray(blob["keys"], np.int32)
        sdf = np.ascontiguousarray(blob["sdf"], np.float32)
        w = np.ascontiguousarray(blob["w"], np.float32)
        rgb = blob.get("rgb")
        wc = blob.get("wc")
        rgb = None if rgb is None else np.ascontiguousarray(rgb, np.uint8)
        wc = None if wc is None else np.ascontiguousarray(wc, np.float32)
        b = _Blob(keys.shape[0], keys.ctypes.data, sdf.ctypes.data, w.ctypes.data,
                  rgb.ctypes.data if rgb is not None else None,
                  wc.ctypes.data if wc is not None else None)
        _check(_lib.dtsdf_import(self._h, ctypes.byref(b)), "dtsdf_import")


class Volume(Map):
    """A view-dependent combined TSDF of a map (Sec. 4): one regular volume that renders, from
    (near) the pose it was combined for, like the six directions it was combined from."""

    def __init__(self, src: Map, brick_capacity: Optional[int] = None,
                 hash_buckets: Optional[int] = None):
        cap = int(brick_capacity if brick_capacity is not None
                  else max(1024, src.params.brick_capacity // 4))
        nb = int(hash_buckets if hash_buckets is not None else src.params.hash_buckets)
        self.params = dataclasses.replace(src.params, sdf_fmt=SDF_F32, w_fmt=W_F32,
                                          brick_capacity=cap, hash_buckets=nb,
                                          dense_lo=None, dense_hi=None)
        h = _V()
        _check(_lib.dtsdf_volume_create(src.handle, cap, nb, ctypes.byref(h)),
               "dtsdf_volume_create")
        self._h = h

    def integrate(self, *args, **kwargs):
        raise TypeError("a combined TSDF is written by combine(), not by integrate()")

    def combine(self, src: Map, cam, T_center, T_frustum=None, margin: float = 0.125,
                only_missing: bool = False, stream=None) -> int:
        """Combine ``src`` for the camera centre of ``T_center`` over the frustum of
        ``T_frustum`` (default: T_center) widened by ``margin`` (see dtsdf_combine)."""
        Tf = T_center if T_frustum is None else T_frustum
        return _check(_lib.dtsdf_combine(src.handle, self._h, _pose(T_center), _pose(Tf),
                                         ctypes.byref(_intr(cam)), margin, int(only_missing),
                                         _stream(stream)), "dtsdf_combine")


class RecombinePolicy:
    """Conditional recombination (Sec. 4, eq. condition_1 .. condition_4), decided by the
    library: boot up, stale state, translation and rotation limits."""

    def __init__(self, boot_frames: int = 5, stale_frames: int = 50,
                 max_translation: float = 0.05, max_angle: float = 0.05 * math.pi / 2):
        self._s = _RecombineState()
        self._s.boot_frames = boot_frames
        self._s.stale_frames = stale_frames
        self._s.max_translation = max_translation
        self._s.max_angle = max_angle

    def decide(self, T_wc) -> bool:
        out = ctypes.c_int32(0)
        _check(_lib.dtsdf_recombine_decide(ctypes.byref(self._s), _pose(T_wc),
                                           ctypes.byref(out)), "dtsdf_recombine_decide")
        return bool(out.value)

    @property
    def last_pose(self) -> np.ndarray:
        return np.array(self._s.last_pose[:]).reshape(4, 4)


def vertex_normal(depth: torch.Tensor, cam, depth_scale: float = 1.0, stream=None):
    """(vertex, normal) as (3, H, W) float32 device tensors."""
    H, W = int(cam.height), int(cam.width)
    v = torch.empty((3, H, W), dtype=torch.float32, device=depth.device)
    n = torch.empty((3, H, W), dtype=torch.float32, device=depth.device)
    _check(_lib.dtsdf_vertex_normal(_dev_ptr(depth, torch.float32, H * W),
                                    ctypes.byref(_intr(cam)), depth_scale,
                                    _dev_ptr(v, torch.float32), _dev_ptr(n, torch.float32),
                                    _stream(stream)), "dtsdf_vertex_normal")
    return v, n


def depth_downsample(depth: torch.Tensor, stream=None) -> torch.Tensor:
    H, W = depth.shape
    out = torch.empty((H // 2, W // 2), dtype=torch.float32, device=depth.device)
    _check(_lib.dtsdf_depth_downsample(_dev_ptr(depth, torch.float32), W, H,
                                       _dev_ptr(out, torch.float32), _stream(stream)),
           "dtsdf_depth_downsample")
    return out


@dataclasses.dataclass
class IcpParams:
    max_dist: float = 0.10
    max_angle_deg: float = 20.0
    weight: int = ICP_W_CONST
    z_min: float = 0.1
    min_inliers_per_dim: int = 64
    compensated: bool = False


@dataclasses.dataclass
class Photo:
    """Photometric term of combined ICP (see dtsdf_photo): live and reference grey images
    (float32 device tensors), the reference intrinsics and the model -> reference transform."""
    live_intensity: torch.Tensor
    ref_intensity: torch.Tensor
    ref_cam: object
    T_ref_model: np.ndarray = dataclasses.field(default_factory=lambda: np.eye(4))
    lam: float = 0.1
    max_error: float = 0.05

    def c_struct(self, live_cam) -> _Photo:
        Hl, Wl = int(live_cam.height), int(live_cam.width)
        Hr, Wr = int(self.ref_cam.height), int(self.ref_cam.width)
        return _Photo(_dev_ptr(self.live_intensity, torch.float32, Hl * Wl),
                      _dev_ptr(self.ref_intensity, torch.float32, Hr * Wr),
                      _intr(self.ref_cam), _pose(self.T_ref_model), self.lam, self.max_error)


@dataclasses.dataclass
class DepthFilterParams:
    """Depth support filter + bilateral depth filter (see dtsdf_depth_filter_params); the
    defaults are the values of Sec. 7 and Sec. 8 (support_rel is not given there)."""
    support_rel: float = 0.02
    min_support: int = 2
    sigma_d: float = 5.0
    sigma_r: float = 0.025
    radius: int = 5


def depth_filter(depth: torch.Tensor, params: DepthFilterParams = DepthFilterParams(),
                 stream=None) -> torch.Tensor:
    """Support-filtered and bilaterally filtered copy of an (H, W) float32 device depth."""
    H, W = int(depth.shape[0]), int(depth.shape[1])
    out = torch.empty((H, W), dtype=torch.float32, device=depth.device)
    p = _DepthFilterParams(params.support_rel, params.min_support, params.sigma_d,
                           params.sigma_r, params.radius)
    _check(_lib.dtsdf_depth_filter(_dev_ptr(depth, torch.float32, H * W), W, H, ctypes.byref(p),
                                   _dev_ptr(out, torch.float32), _stream(stream)),
           "dtsdf_depth_filter")
    return out


def normal_filter(normal: torch.Tensor, sigma_d: float = 2.5, sigma_r_deg: float = 5.0,
                  radius: int = 5, stream=None) -> torch.Tensor:
    """Bilaterally filtered copy of a planar (3, H, W) float32 device normal map."""
    H, W = int(normal.shape[1]), int(normal.shape[2])
    out = torch.empty_like(normal)
    _check(_lib.dtsdf_normal_filter(_dev_ptr(normal, torch.float32, 3 * H * W), W, H, sigma_d,
                                    sigma_r_deg, radius, _dev_ptr(out, torch.float32),
                                    _stream(stream)), "dtsdf_normal_filter")
    return out


@dataclasses.dataclass
class Preprocess:
    """Live-frame preprocessing of the registration (Sec. 7): the depth filter before the
    pyramid and the bilateral normal filter on every level's cross-product normals."""
    depth: Optional[DepthFilterParams] = dataclasses.field(default_factory=DepthFilterParams)
    normal_sigma_d: float = 2.5
    normal_sigma_r_deg: float = 5.0
    normal_radius: int = 5          # 0: no normal filter


def _live_levels(live_depth, live_cam, L, depth_scale, pre, stream):
    d0 = live_depth
    if pre is not None and pre.depth is not None:
        d0 = depth_filter(live_depth, pre.depth, stream=stream)
    pyr = [d0]
    for _ in range(1, L):
        pyr.append(depth_downsample(pyr[-1], stream=stream))
    out = []
    for l in range(L):
        cam_l = level_camera(live_cam, l)
        v, n = vertex_normal(pyr[l], cam_l, depth_scale, stream=stream)
        if pre is not None and pre.normal_radius > 0:
            n = normal_filter(n, pre.normal_sigma_d, pre.normal_sigma_r_deg, pre.normal_radius,
                              stream=stream)
        out.append((cam_l, v, n))
    return out


def depth_error(rendered: torch.Tensor, measured: torch.Tensor, stream=None):
    """Post-fusion error (Sec. 8): (mean |rendered - measured| over pixels where both are
    valid, that pixel count)."""
    H, W = int(rendered.shape[0]), int(rendered.shape[1])
    if tuple(measured.shape) != (H, W):
        raise ValueError("depth images differ in shape")
    out = torch.zeros(2, dtype=torch.float64, device=rendered.device)
    _check(_lib.dtsdf_depth_error(_dev_ptr(rendered, torch.float32, H * W),
                                  _dev_ptr(measured, torch.float32, H * W), W, H,
                                  _dev_ptr(out, torch.float64), _stream(stream)),
           "dtsdf_depth_error")
    s, n = out.cpu().tolist()
    return (s / n if n else 0.0), int(n)


def intensity(rgb: torch.Tensor, stream=None) -> torch.Tensor:
    """Grey values in [0, 1] of an (H, W, 3) uint8 device image."""
    H, W = int(rgb.shape[0]), int(rgb.shape[1])
    out = torch.empty((H, W), dtype=torch.float32, device=rgb.device)
    _check(_lib.dtsdf_intensity(_dev_ptr(rgb, torch.uint8, H * W * 3), W, H,
                                _dev_ptr(out, torch.float32), _stream(stream)), "dtsdf_intensity")
    return out


def intensity_downsample(img: torch.Tensor, stream=None) -> torch.Tensor:
    H, W = img.shape
    out = torch.empty((H // 2, W // 2), dtype=torch.float32, device=img.device)
    _check(_lib.dtsdf_intensity_downsample(_dev_ptr(img, torch.float32), W, H,
                                           _dev_ptr(out, torch.float32), _stream(stream)),
           "dtsdf_intensity_downsample")
    return out


def _icp_images(live_vertex, live_normal, live_cam, model_vertex, model_normal, model_mask,
                model_cam, params):
    Hl, Wl = int(live_cam.height), int(live_cam.width)
    Hm, Wm = int(model_cam.height), int(model_cam.width)
    live = _Image(_dev_ptr(live_vertex, torch.float32, 3 * Hl * Wl),
                  _dev_ptr(live_normal, torch.float32, 3 * Hl * Wl), None, _intr(live_cam))
    model = _Image(_dev_ptr(model_vertex, torch.float32, 3 * Hm * Wm),
                   _dev_ptr(model_normal, torch.float32, 3 * Hm * Wm),
                   _dev_ptr(model_mask, torch.uint8, Hm * Wm) if model_mask is not None else None,
                   _intr(model_cam))
    p = _IcpParams(params.max_dist, params.max_angle_deg, params.weight, params.z_min,
                   params.min_inliers_per_dim, int(params.compensated))
    return live, model, p


def icp_step(live_vertex: torch.Tensor, live_normal: torch.Tensor, live_cam,
             model_vertex: torch.Tensor, model_normal: torch.Tensor,
             model_mask: Optional[torch.Tensor], model_cam, T_model_live, dim: int = 6,
             params: IcpParams = IcpParams(), stream=None, photo: Optional[Photo] = None):
    """One ICP Gauss-Newton step (with ``photo``: combined geometric + photometric);
    returns (status, updated T (4x4), result dict)."""
    live, model, p = _icp_images(live_vertex, live_normal, live_cam, model_vertex,
                                 model_normal, model_mask, model_cam, params)
    T = _pose(T_model_live)
    r = _IcpResult()
    ph = ctypes.byref(photo.c_struct(live_cam)) if photo is not None else None
    status = _lib.icp_step_rgb(ctypes.byref(live), ctypes.byref(model), ph, dim,
                               ctypes.byref(p), T, ctypes.byref(r), _stream(stream))
    _check(status, "icp_step", allow=(E_DEGENERATE,))
    res = dict(xi=np.array(r.xi[:dim]), H=np.array(r.H[:dim * dim]).reshape(dim, dim),
               g=np.array(r.g[:dim]), error=r.error, inliers=r.inliers, step_norm=r.step_norm,
               photometric=r.photometric)
    return status, np.array(T[:]).reshape(4, 4), res


class LmState:
    """Levenberg-Marquardt state of one registration run (see dtsdf_lm_state): set the prior
    pose and tau, then call icp_step_lm until the step is small; the result is T_acc."""

    def __init__(self, T0, tau: float = 1e-3):
        self.c = _LmState()
        self.c.T[:] = [float(v) for v in np.asarray(T0, np.float64).ravel()]
        self.c.T_acc[:] = self.c.T[:]
        self.c.tau = tau
        self.c.nu = 2.0

    @property
    def T(self) -> np.ndarray:
        return np.array(self.c.T[:]).reshape(4, 4)

    @property
    def T_acc(self) -> np.ndarray:
        return np.array(self.c.T_acc[:]).reshape(4, 4)

    @property
    def mu(self) -> float:
        return self.c.mu

    @property
    def accepted(self) -> bool:
        return bool(self.c.accepted)


def icp_step_lm(live_vertex: torch.Tensor, live_normal: torch.Tensor, live_cam,
                model_vertex: torch.Tensor, model_normal: torch.Tensor,
                model_mask: Optional[torch.Tensor], model_cam, state: LmState, dim: int = 7,
                params: IcpParams = IcpParams(), stream=None, photo: Optional[Photo] = None):
    """One Levenberg-Marquardt ICP iteration (Sec. 7) at state.T; updates ``state`` and
    returns (status, result dict)."""
    live, model, p = _icp_images(live_vertex, live_normal, live_cam, model_vertex,
                                 model_normal, model_mask, model_cam, params)
    r = _IcpResult()
    ph = ctypes.byref(photo.c_struct(live_cam)) if photo is not None else None
    status = _lib.icp_step_lm(ctypes.byref(live), ctypes.byref(model), ph, dim, ctypes.byref(p),
                              ctypes.byref(state.c), ctypes.byref(r), _stream(stream))
    _check(status, "icp_step_lm", allow=(E_DEGENERATE,))
    res = dict(xi=np.array(r.xi[:dim]), H=np.array(r.H[:dim * dim]).reshape(dim, dim),
               g=np.array(r.g[:dim]), error=r.error, inliers=r.inliers, step_norm=r.step_norm,
               photometric=r.photometric)
    return status, res


def icp_lm(live_depth: torch.Tensor, live_cam, model_levels, T0, dim: int = 7,
           iters=(10, 5, 4), params: IcpParams = IcpParams(), tau: float = 1e-3,
           min_step: float = 1e-6, depth_scale: float = 1.0, stream=None,
           preprocess: Optional[Preprocess] = None):
    """Coarse-to-fine ICP solved by Levenberg-Marquardt with Madsen's damping (Sec. 7); the
    damping restarts at every level and each level starts from the previous level's
    accepted pose.  ``preprocess`` filters the live frame first (Sec. 7)."""
    L = len(model_levels)
    live = _live_levels(live_depth, live_cam, L, depth_scale, preprocess, stream)
    T = np.array(T0, np.float64)
    log = []
    for l in reversed(range(L)):
        cam_l, v, n = live[l]
        mv, mn, mm, mcam = model_levels[l]
        st = LmState(T, tau)
        for _ in range(iters[l]):
            status, res = icp_step_lm(v, n, cam_l, mv, mn, mm, mcam, st, dim, params, stream)
            if status != OK:
                log.append(dict(level=l, status="degenerate", inliers=res["inliers"],
                                err=res["error"]))
                break
            log.append(dict(level=l, inliers=res["inliers"], err=res["error"],
                            accepted=st.accepted, mu=st.mu, step=res["step_norm"]))
            if res["step_norm"] < min_step:
                break
        T = st.T_acc
    return T, log


@dataclasses.dataclass
class IcpRequest:
    """One request of icp_step_batch: device images plus device pose / flag / result."""
    live_vertex: torch.Tensor
    live_normal: torch.Tensor
    live_cam: object
    model_vertex: torch.Tensor
    model_normal: torch.Tensor
    model_mask: Optional[torch.Tensor]
    model_cam: object
    pose: torch.Tensor                 # float64 (4, 4) device tensor, updated in place
    active: Optional[torch.Tensor]     # int32 (1,) device tensor or None
    result: Optional[torch.Tensor]     # uint8 (ICP_RESULT_BYTES,) device tensor or None
    dim: int = 6
    params: IcpParams = dataclasses.field(default_factory=IcpParams)
    min_step: float = 0.0


def icp_request_struct(q: IcpRequest) -> _IcpReq:
    """The C descriptor of one batched ICP request (kept by callers that reuse it)."""
    r = _IcpReq()
    Hl, Wl = int(q.live_cam.height), int(q.live_cam.width)
    Hm, Wm = int(q.model_cam.height), int(q.model_cam.width)
    r.live = _Image(_dev_ptr(q.live_vertex, torch.float32, 3 * Hl * Wl),
                    _dev_ptr(q.live_normal, torch.float32, 3 * Hl * Wl), None, _intr(q.live_cam))
    r.model = _Image(_dev_ptr(q.model_vertex, torch.float32, 3 * Hm * Wm),
                     _dev_ptr(q.model_normal, torch.float32, 3 * Hm * Wm),
                     _dev_ptr(q.model_mask, torch.uint8, Hm * Wm)
                     if q.model_mask is not None else None, _intr(q.model_cam))
    r.dim = q.dim
    p = q.params
    r.params = _IcpParams(p.max_dist, p.max_angle_deg, p.weight, p.z_min,
                          p.min_inliers_per_dim, int(p.compensated))
    r.pose = _dev_ptr(q.pose, torch.float64, 16)
    r.active = _dev_ptr(q.active, torch.int32, 1) if q.active is not None else None
    r.min_step = q.min_step
    r.result = _dev_ptr(q.result, torch.uint8, ICP_RESULT_BYTES) if q.result is not None else None
    r.photo = None
    return r


def icp_step_batch_structs(structs, stream=None) -> None:
    """icp_step_batch over prebuilt descriptors (see icp_request_struct)."""
    n = len(structs)
    reqs = (_IcpReq * n)(*structs)
    _check(_lib.icp_step_batch(n, reqs, _stream(stream)), "icp_step_batch")


def icp_step_batch(requests, stream=None) -> None:
    icp_step_batch_structs([icp_request_struct(q) for q in requests], stream)


def icp_step_batch_iters(requests, iterations: int, stream=None) -> None:
    """`iterations` steps of icp_step_batch from one upload of the requests."""
    structs = [icp_request_struct(q) for q in requests]
    n = len(structs)
    reqs = (_IcpReq * n)(*structs)
    _check(_lib.icp_step_batch_iters(n, reqs, int(iterations), _stream(stream)),
           "icp_step_batch_iters")


def icp_step_batch_iters_noalloc(requests, iterations: int, stream=None) -> None:
    """icp_step_batch_iters without any allocation (at most NOALLOC_MAX_REQUESTS requests;
    calls on one GPU must not overlap)."""
    structs = [icp_request_struct(q) for q in requests]
    n = len(structs)
    reqs = (_IcpReq * max(n, 1))(*structs)
    _check(_lib.icp_step_batch_iters_noalloc(n, reqs, int(iterations), _stream(stream)),
           "icp_step_batch_iters_noalloc")


def decode_result(raw: torch.Tensor, dim: int = 7) -> dict:
    """The dtsdf_icp_result a batched ICP step wrote to device memory."""
    r = _IcpResult.from_buffer_copy(bytes(raw.cpu().numpy()))
    return dict(xi=np.array(r.xi[:dim]), H=np.array(r.H[:dim * dim]).reshape(dim, dim),
                g=np.array(r.g[:dim]), error=r.error, inliers=r.inliers,
                step_norm=r.step_norm, status=r.status)


def icp(live_depth: torch.Tensor, live_cam, model_levels, T0, dim: int = 6,
        iters=(10, 5, 4), params: IcpParams = IcpParams(), min_step: float = 1e-6,
        depth_scale: float = 1.0, stream=None, live_rgb: Optional[torch.Tensor] = None,
        ref_levels=None, T_ref_model=None, lam: float = 0.1, max_error=(0.05, 0.175, 0.175),
        preprocess: Optional[Preprocess] = None):
    """Coarse-to-fine ICP: model_levels[l] = (vertex, normal, mask, cam) at level l.
    ``iters`` lists fine-to-coarse iteration counts; levels run coarse to fine.
    With ``live_rgb`` and ``ref_levels`` ([(grey image, cam)] per level) the steps are
    combined geometric + photometric (Sec. 5.2, 5.3); ``T_ref_model`` maps the model camera to
    the reference camera (identity: frame-to-frame / frame-to-render).  ``preprocess``
    filters the live frame first (Sec. 7)."""
    L = len(model_levels)
    live = _live_levels(live_depth, live_cam, L, depth_scale, preprocess, stream)
    ipyr = None
    if live_rgb is not None:
        ipyr = [intensity(live_rgb, stream=stream)]
        for _ in range(1, L):
            ipyr.append(intensity_downsample(ipyr[-1], stream=stream))
    Tref = np.eye(4) if T_ref_model is None else np.asarray(T_ref_model, np.float64)
    T = np.array(T0, np.float64)
    log = []
    for l in reversed(range(L)):
        cam_l, v, n = live[l]
        mv, mn, mm, mcam = model_levels[l]
        photo = None
        if ipyr is not None:
            ri, rcam = ref_levels[l]
            photo = Photo(ipyr[l], ri, rcam, Tref, lam, max_error[l])
        for _ in range(iters[l]):
            status, T_new, res = icp_step(v, n, cam_l, mv, mn, mm, mcam, T, dim, params, stream,
                                          photo=photo)
            if status != OK:
                log.append(dict(level=l, status="degenerate", inliers=res["inliers"],
                                err=res["error"]))
                break
            T = T_new
            log.append(dict(level=l, inliers=res["inliers"], err=res["error"],
                            step=res["step_norm"], photometric=res["photometric"], H=res["H"]))
            if res["step_norm"] < min_step:
                break
    return T, log


def render_levels(src, cam, T_wc, levels: int = 3, z_near: float = 0.2, z_far: float = 10.0,
                  stream=None):
    """Model pyramid for ICP: vertex, normal and mask of ``src`` (a Map or a Volume) at pose
    T_wc for pyramid levels 0 .. levels-1, all rendered in one batched launch (the levels'
    tails overlap); each level equals src.render of that level bitwise.  Returns
    [(vertex, normal, mask, cam_l)]."""
    dev = torch.device("cuda", torch.cuda.current_device())
    views, out = [], []
    for l in range(levels):
        c = level_camera(cam, l)
        H, W = int(c.height), int(c.width)
        o = dict(vertex=torch.empty((3, H, W), dtype=torch.float32, device=dev),
                 normal=torch.empty((3, H, W), dtype=torch.float32, device=dev),
                 mask=torch.empty((H, W), dtype=torch.uint8, device=dev))
        views.append((c, T_wc, z_near, z_far, o))
        out.append((o["vertex"], o["normal"], o["mask"], c))
    src.render_batch(views, stream=stream)
    return out


def icp_device(live_depth: torch.Tensor, live_cam, model_levels, T0, dim: int = 6,
               iters=(10, 5, 4), params: IcpParams = IcpParams(), min_step: float = 1e-6,
               depth_scale: float = 1.0, stream=None, preprocess: Optional[Preprocess] = None,
               live_rgb: Optional[torch.Tensor] = None, ref_levels=None, T_ref_model=None,
               lam: float = 0.1, max_error=(0.05, 0.175, 0.175)):
    """The coarse-to-fine ICP of icp() with the pose, the convergence flag and the sums kept
    in device memory: each level's iterations are enqueued by one icp_step_batch_iters call
    without a host wait (a converged or degenerate level skips its remaining iterations on
    the device), and the pose is copied back once.  Same steps, same result as icp()."""
    L = len(model_levels)
    live = _live_levels(live_depth, live_cam, L, depth_scale, preprocess, stream)
    ipyr = None
    if live_rgb is not None:
        ipyr = [intensity(live_rgb, stream=stream)]
        for _ in range(1, L):
            ipyr.append(intensity_downsample(ipyr[-1], stream=stream))
    Tref = np.eye(4) if T_ref_model is None else np.asarray(T_ref_model, np.float64)
    dev = live_depth.device
    pose = torch.tensor(np.asarray(T0, np.float64), dtype=torch.float64, device=dev)
    active = torch.ones(1, dtype=torch.int32, device=dev)
    reqs = (_IcpReq * L)()
    photos = []       # kept alive until the call has copied them
    for l in range(L):
        cam_l, v, n = live[l]
        mv, mn, mm, mcam = model_levels[l]
        reqs[l] = icp_request_struct(IcpRequest(v, n, cam_l, mv, mn, mm, mcam, pose, active,
                                                None, dim, params, min_step))
        if ipyr is not None:
            ri, rcam = ref_levels[l]
            photos.append(Photo(ipyr[l], ri, rcam, Tref, lam, max_error[l]).c_struct(cam_l))
            reqs[l].photo = ctypes.addressof(photos[-1])
    its = (ctypes.c_int32 * L)(*[int(i) for i in iters])
    _check(_lib.dtsdf_icp_pyramid(L, reqs, its, _stream(stream)), "dtsdf_icp_pyramid")
    return pose.cpu().numpy()


@dataclasses.dataclass(frozen=True)
class LevelCamera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float


def level_camera(cam, l: int):
    """Intrinsics of pyramid level l (dtsdf_level_intrinsics); level 0 is `cam` itself."""
    if l == 0:
        return cam
    o = _Intr()
    _check(_lib.dtsdf_level_intrinsics(ctypes.byref(_intr(cam)), int(l), ctypes.byref(o)),
           "dtsdf_level_intrinsics")
    return LevelCamera(o.width, o.height, o.fx, o.fy, o.cx, o.cy)
