"""Plain FP64 CPU oracle of the Directional TSDF hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark may import this
module.  It shares no code with the HIP library; both sides only consume the seeded inputs of
``synth``.

* Integration and rendering (Sec. 3, Sec. 4) live in ``dtsdf_oracle.cpp`` (plain C++ in
  double precision) and are wrapped here through ctypes.
* Registration (Sec. 5 and Sec. 6) is written here with numpy in float64: projective data
  association, the point-to-plane residual (eq. geometric_ICP), its Jacobian
  (eq. ICP_geometric_dx; Sim(3): eq. sim3_derivative), the normal equations
  (eq. ICP_Hessian), the Cholesky solve (eq. ICP_solution) and the left-multiplied update
  (eq. deltaT_update); the photometric terms of combined ICP (eq. combined_icp) against a
  reference grey image with a keyframe offset (eq. keyframe_icp and its derivative);
  Levenberg-Marquardt with Madsen's damping (Sec. 7) and scale anchoring (Sec. 6).  The
  exponential maps are the matrix exponential of the 4x4 generator (scipy.linalg.expm), the
  plain definition of exp on se(3) and sim(3).
* Input preprocessing (Sec. 7, Sec. 8 parameters): the depth support filter and the
  bilateral depth and normal filters by their definitions; the post-fusion error (Sec. 8).

Parameters are passed as float32-representable values (``f32``) so that both implementations
compare against exactly the same thresholds.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import Optional, Sequence

import numpy as np
import scipy.linalg

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "dtsdf_oracle.cpp")


def build(force: bool = False) -> str:
    """Compile the C++ oracle (g++, OpenMP) next to its source."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c++17",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        _declare(_lib)
    return _lib


def f32(x: float) -> float:
    return float(np.float32(x))


class _Params(ctypes.Structure):
    _fields_ = [("voxel", ctypes.c_double), ("tau", ctypes.c_double),
                ("theta", ctypes.c_double), ("w_carve", ctypes.c_double),
                ("w_max", ctypes.c_double), ("w_min", ctypes.c_double),
                ("step", ctypes.c_double), ("dense", ctypes.c_int32),
                ("dense_lo", ctypes.c_int32 * 3), ("dense_hi", ctypes.c_int32 * 3),
                ("with_color", ctypes.c_int32), ("single_direction", ctypes.c_int32),
                ("sdf_fmt", ctypes.c_int32), ("w_fmt", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_int64), ("borderline_req", ctypes.c_int64),
                ("new_bricks", ctypes.c_int64), ("updated", ctypes.c_int64),
                ("carved", ctypes.c_int64)]


class _RenderCfg(ctypes.Structure):
    _fields_ = [("z_near", ctypes.c_double), ("z_far", ctypes.c_double),
                ("eps_f", ctypes.c_double), ("eps_x", ctypes.c_double),
                ("eps_s", ctypes.c_double), ("eps_root", ctypes.c_double),
                ("classify", ctypes.c_int32), ("eps_n", ctypes.c_double),
                ("eps_c", ctypes.c_double)]


_P = ctypes.c_void_p


def _declare(L):
    L.orc_create.restype = _P
    L.orc_create.argtypes = [ctypes.POINTER(_Params)]
    L.orc_destroy.argtypes = [_P]
    L.orc_num_bricks.restype = ctypes.c_int64
    L.orc_num_bricks.argtypes = [_P]
    L.orc_integrate.argtypes = [_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double, _P,
                                ctypes.c_double, ctypes.POINTER(_Stats), _P]
    L.orc_requests.restype = ctypes.c_int64
    L.orc_requests.argtypes = [_P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double, _P,
                               ctypes.c_double, _P, _P, _P, ctypes.c_int64, _P]
    L.orc_recycle.restype = ctypes.c_int64
    L.orc_recycle.argtypes = [_P, ctypes.c_double]
    L.orc_export.restype = ctypes.c_int64
    L.orc_export.argtypes = [_P] * 7
    L.orc_import.argtypes = [_P, ctypes.c_int64, _P, _P, _P, _P, _P]
    L.orc_render.argtypes = [_P, ctypes.c_int64, _P, _P, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double, ctypes.c_double, _P, ctypes.POINTER(_RenderCfg),
                             _P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.orc_eval.argtypes = [_P, ctypes.c_int64, _P, _P, _P, _P, _P]
    L.orc_shade.argtypes = [_P, ctypes.c_int64, _P, _P, _P, _P, _P]
    L.orc_brick_key.argtypes = [_P, ctypes.c_int64, _P]
    L.orc_combine.argtypes = [_P, _P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                              ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    L.orc_num_threads.restype = ctypes.c_int
    L.orc_w_dir.restype = ctypes.c_double
    L.orc_w_dir.argtypes = [ctypes.POINTER(_Params), _P, ctypes.c_int]


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "arrays passed to the oracle must be contiguous"
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------------------
# Map parameters.  Values the paper does not give are proposals (see the design notes).
# ----------------------------------------------------------------------------------------

@dataclasses.dataclass
class MapParams:
    voxel: float
    tau: float
    theta: float = math.pi / 3.0
    w_carve: float = 0.1
    w_max: float = 63.75
    w_min: float = 1e-4
    step: Optional[float] = None            # default: half a voxel
    dense_lo: Optional[Sequence[int]] = None
    dense_hi: Optional[Sequence[int]] = None
    with_color: bool = True
    single_direction: bool = False
    sdf_fmt: int = 0            # 0 float, 1 float16, 2 int16 scaled by the truncation
    w_fmt: int = 0              # 0 float, 1 uint8 code q, w = q^2 / 1024

    def c_struct(self) -> _Params:
        p = _Params()
        p.voxel = f32(self.voxel)
        p.tau = f32(self.tau)
        p.theta = f32(self.theta)
        p.w_carve = f32(self.w_carve)
        p.w_max = f32(self.w_max)
        p.w_min = f32(self.w_min)
        p.step = f32(self.step if self.step is not None else 0.5 * self.voxel)
        p.dense = 1 if self.dense_lo is not None else 0
        for k in range(3):
            p.dense_lo[k] = int(self.dense_lo[k]) if self.dense_lo is not None else 0
            p.dense_hi[k] = int(self.dense_hi[k]) if self.dense_hi is not None else 0
        p.with_color = int(self.with_color)
        p.single_direction = int(self.single_direction)
        p.sdf_fmt = int(self.sdf_fmt)
        p.w_fmt = int(self.w_fmt)
        return p


def num_threads() -> int:
    return int(lib().orc_num_threads())


def w_dir(params: MapParams, n: Sequence[float], d: int) -> float:
    """Direction membership weight of unit normal ``n`` for direction ``d`` (X+,X-,Y+,...)."""
    cp = params.c_struct()
    nn = np.ascontiguousarray(n, np.float64)
    return lib().orc_w_dir(ctypes.byref(cp), _ptr(nn), int(d))


@dataclasses.dataclass
class RenderOut:
    depth: np.ndarray
    vertex: np.ndarray
    normal: np.ndarray
    rgba: np.ndarray
    mask: np.ndarray
    flags: np.ndarray
    khit: np.ndarray
    thit: np.ndarray
    touched: Optional[np.ndarray] = None


# Grazing flag bits returned by render()
NEAR_ZERO, NEAR_FACE, BRANCH, AMBIGUOUS, ROOT_FACE, ROOT_BRANCH, ROOT_SHADE = \
    1, 2, 4, 8, 16, 32, 64


class OracleMap:
    """A DTSDF map held by the C++ oracle."""

    def __init__(self, params: MapParams):
        self.params = params
        self._cp = params.c_struct()
        self._h = lib().orc_create(ctypes.byref(self._cp))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    @property
    def num_bricks(self) -> int:
        return int(lib().orc_num_bricks(self._h))

    def integrate(self, depth: np.ndarray, rgb: Optional[np.ndarray], cam, T_wc: np.ndarray,
                  depth_scale: float = 1.0, normals: Optional[np.ndarray] = None) -> dict:
        """Fuse one frame; ``normals`` (H, W, 3 camera frame, zero = none) replaces the
        cross-product normals (e.g. filtered ones, Sec. 7)."""
        d = np.ascontiguousarray(depth, np.float32)
        c = None if rgb is None else np.ascontiguousarray(rgb, np.uint8)
        T = np.ascontiguousarray(T_wc, np.float64)
        nrm = None if normals is None else np.ascontiguousarray(normals, np.float64)
        st = _Stats()
        lib().orc_integrate(self._h, _ptr(d), _ptr(c), d.shape[1], d.shape[0], cam.fx, cam.fy,
                            cam.cx, cam.cy, _ptr(T), f32(depth_scale), ctypes.byref(st),
                            _ptr(nrm))
        return {k: getattr(st, k) for k, _ in _Stats._fields_}

    def requests(self, depth: np.ndarray, cam, T_wc: np.ndarray, depth_scale: float = 1.0,
                 normals: Optional[np.ndarray] = None):
        """(keys n x 4, borderline flags, allocating flags) of one frame's block requests."""
        d = np.ascontiguousarray(depth, np.float32)
        T = np.ascontiguousarray(T_wc, np.float64)
        cap = d.size * 6 * 64
        keys = np.zeros((cap, 4), np.int32)
        border = np.zeros(cap, np.uint8)
        alloc = np.zeros(cap, np.uint8)
        nrm = None if normals is None else np.ascontiguousarray(normals, np.float64)
        n = lib().orc_requests(self._h, _ptr(d), d.shape[1], d.shape[0], cam.fx, cam.fy, cam.cx,
                               cam.cy, _ptr(T), f32(depth_scale), _ptr(keys), _ptr(border),
                               _ptr(alloc), cap, _ptr(nrm))
        assert n <= cap
        return keys[:n], border[:n], alloc[:n]

    def recycle(self, t_free: float = 0.9) -> int:
        """Recycling of bricks without surface (Sec. 3): removes every brick whose observed
        voxels all hold values >= t_free (or that has none); returns how many."""
        return int(lib().orc_recycle(self._h, f32(t_free)))

    def export(self) -> dict:
        n = self.num_bricks
        out = dict(keys=np.zeros((n, 4), np.int32), sdf=np.zeros((n, 512), np.float32),
                   w=np.zeros((n, 512), np.float32), rgb=np.zeros((n, 512, 3), np.uint8),
                   wc=np.zeros((n, 512), np.float32), border=np.zeros((n, 512), np.uint8))
        lib().orc_export(self._h, _ptr(out["keys"]), _ptr(out["sdf"]), _ptr(out["w"]),
                         _ptr(out["rgb"]), _ptr(out["wc"]), _ptr(out["border"]))
        return out

    def load(self, blob: dict) -> None:
        keys = np.ascontiguousarray(blob["keys"], np.int32)
        sdf = np.ascontiguousarray(blob["sdf"], np.float32)
        w = np.ascontiguousarray(blob["w"], np.float32)
        rgb = blob.get("rgb")
        wc = blob.get("wc")
        rgb = None if rgb is None else np.ascontiguousarray(rgb, np.uint8)
        wc = None if wc is None else np.ascontiguousarray(wc, np.float32)
        lib().orc_import(self._h, keys.shape[0], _ptr(keys), _ptr(sdf), _ptr(w), _ptr(rgb),
                         _ptr(wc))

    def render(self, cam, T_wc: np.ndarray, *, pixels: Optional[np.ndarray] = None,
               z_near: float = 0.2, z_far: float = 10.0, eps_f: float = 1e-5,
               eps_x: float = 1e-6, eps_s: float = 1e-5, eps_root: float = 2e-6,
               eps_n_deg: float = 0.25, eps_c: float = 0.5,
               classify: bool = True, touched: bool = False) -> RenderOut:
        """Render all pixels (or the (n,2) array of (u, v) ``pixels``).

        With ``classify`` the grazing flags are computed (eps_f: |f| near zero; eps_x: voxel
        distance to a cell face; eps_s: margin on thresholded weight factors; eps_root: metres
        along the ray within which the root is taken as known; eps_n_deg, eps_c: the turn of
        the normal and the change of a colour channel within eps_root of the root above which
        the shading counts as not fixed by it); without it only the plain render runs."""
        if pixels is None:
            vv, uu = np.mgrid[0:cam.height, 0:cam.width]
            pixels = np.stack([uu.ravel(), vv.ravel()], axis=1)
        pixels = np.asarray(pixels)
        us = np.ascontiguousarray(pixels[:, 0], np.int32)
        vs = np.ascontiguousarray(pixels[:, 1], np.int32)
        n = us.shape[0]
        o = RenderOut(depth=np.zeros(n), vertex=np.zeros((n, 3)), normal=np.zeros((n, 3)),
                      rgba=np.zeros((n, 4), np.uint8), mask=np.zeros(n, np.uint8),
                      flags=np.zeros(n, np.uint8), khit=np.zeros(n, np.int64),
                      thit=np.zeros(n))
        if touched:
            o.touched = np.zeros(self.num_bricks, np.uint8)
        cfg = _RenderCfg(f32(z_near), f32(z_far), eps_f, eps_x, eps_s, eps_root, int(classify),
                         math.radians(eps_n_deg), eps_c)
        T = np.ascontiguousarray(T_wc, np.float64)
        lib().orc_render(self._h, n, _ptr(us), _ptr(vs), cam.fx, cam.fy, cam.cx, cam.cy,
                         _ptr(T), ctypes.byref(cfg), _ptr(o.depth), _ptr(o.vertex),
                         _ptr(o.normal), _ptr(o.rgba), _ptr(o.mask), _ptr(o.flags),
                         _ptr(o.khit), _ptr(o.thit), _ptr(o.touched))
        return o

    def eval(self, xs: np.ndarray, rs: np.ndarray):
        """Combined SDF f at world points xs (n,3) for unit rays rs (n,3): (f, defined, fallback)."""
        xs = np.ascontiguousarray(xs, np.float64)
        rs = np.ascontiguousarray(np.broadcast_to(rs, xs.shape), np.float64)
        n = xs.shape[0]
        f = np.zeros(n)
        d = np.zeros(n, np.uint8)
        fb = np.zeros(n, np.uint8)
        lib().orc_eval(self._h, n, _ptr(xs), _ptr(rs), _ptr(f), _ptr(d), _ptr(fb))
        return f, d.astype(bool), fb.astype(bool)

    def shade(self, xs: np.ndarray, rs: np.ndarray):
        """Shading outputs at world points xs (n,3) for unit rays rs (n,3): world-frame unit
        normal (n,3), unrounded colour (n,3), normal present (n,), colour present (n,)."""
        xs = np.ascontiguousarray(xs, np.float64)
        rs = np.ascontiguousarray(np.broadcast_to(rs, xs.shape), np.float64)
        n = xs.shape[0]
        nrm, rgb, has = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(n, np.uint8)
        lib().orc_shade(self._h, n, _ptr(xs), _ptr(rs), _ptr(nrm), _ptr(rgb), _ptr(has))
        return nrm, rgb, (has & 1) != 0, (has & 2) != 0

    def combine(self, src: "OracleMap", cam, T_center: np.ndarray,
                T_frustum: Optional[np.ndarray] = None, margin: float = 0.125,
                only_missing: bool = False, eps_s: float = 1e-5, eps_edge: float = 1e-6):
        """Write into this single-direction map the view-dependent combined TSDF of ``src``
        (Sec. 4): the combined SDF of every voxel centre in the frustum of ``T_frustum``
        (image widened by ``margin`` of its size per side) for the camera centre of
        ``T_center``.  ``only_missing``: evaluate only voxels of that frustum holding no value
        (voxels seen for the first time) and keep the rest."""
        assert self.params.single_direction, "the combined TSDF is a single-direction map"
        Tc = np.ascontiguousarray(T_center, np.float64)
        Tf = Tc if T_frustum is None else np.ascontiguousarray(T_frustum, np.float64)
        lib().orc_combine(src._h, self._h, _ptr(Tc), _ptr(Tf), int(cam.width), int(cam.height),
                          cam.fx, cam.fy, cam.cx, cam.cy, float(margin), int(only_missing),
                          float(eps_s), float(eps_edge))

    def brick_key(self, i: int) -> np.ndarray:
        k = np.zeros(4, np.int32)
        lib().orc_brick_key(self._h, int(i), _ptr(k))
        return k


# ----------------------------------------------------------------------------------------
# Conditional recombination of the combined TSDF (Sec. 4, eq. condition_1 .. condition_4)
# ----------------------------------------------------------------------------------------

def rotation_angle(R: np.ndarray) -> float:
    """Geodesic angle of a rotation: |log R|_F / sqrt(2) (principal matrix logarithm)."""
    L = scipy.linalg.logm(np.asarray(R, np.float64))
    return float(np.linalg.norm(np.real(L)) / math.sqrt(2.0))


class RecombinePolicy:
    """Decides per frame whether the combined TSDF is recomputed.

    Frame k (counted from 0) triggers a recombination if k < boot_frames (boot up), more than
    stale_frames frames have passed since the last recombination (stale state), or its pose
    differs from the pose of the last recombination by more than max_translation metres or
    max_angle radians of rotation."""

    def __init__(self, boot_frames: int = 5, stale_frames: int = 50,
                 max_translation: float = 0.05, max_angle: float = 0.05 * math.pi / 2):
        self.boot_frames = boot_frames
        self.stale_frames = stale_frames
        self.max_translation = max_translation
        self.max_angle = max_angle
        self.frames = 0
        self.since = 0
        self.last = None

    def decide(self, T: np.ndarray) -> bool:
        T = np.asarray(T, np.float64)
        need = self.last is None or self.frames < self.boot_frames or \
            self.since > self.stale_frames
        if not need:
            dt = float(np.linalg.norm(T[:3, 3] - self.last[:3, 3]))
            da = rotation_angle(self.last[:3, :3].T @ T[:3, :3])
            need = dt > self.max_translation or da > self.max_angle
        self.frames += 1
        if need:
            self.since = 1
            self.last = T.copy()
        else:
            self.since += 1
        return need


# ----------------------------------------------------------------------------------------
# Registration: point-to-plane ICP in SE(3) and Sim(3) (Sec. 5, Sec. 6), numpy float64
# ----------------------------------------------------------------------------------------

def hat(w: np.ndarray) -> np.ndarray:
    """The wedge operator of Sec. 5.3 (eq. wedge_operator)."""
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def generator(xi: np.ndarray) -> np.ndarray:
    """4x4 Lie-algebra matrix of xi = (nu, omega) in se(3) or (nu, omega, sigma) in sim(3)."""
    G = np.zeros((4, 4))
    G[:3, :3] = hat(xi[3:6])
    if len(xi) == 7:
        G[:3, :3] += xi[6] * np.eye(3)
    G[:3, 3] = xi[:3]
    return G


def exp_map(xi: np.ndarray) -> np.ndarray:
    """exp: se(3) -> SE(3) or sim(3) -> Sim(3) as the matrix exponential of the generator.

    For sim(3) this yields [[e^sigma exp(omega^), V nu], [0, 1]] (Sec. 6) with
    V = int_0^1 e^(sigma u) exp(u omega^) du, the matrix the paper leaves undefined."""
    return scipy.linalg.expm(generator(np.asarray(xi, np.float64)))


def depth_pyramid(depth: np.ndarray, levels: int):
    """Level l+1 pixel = mean of the 2x2 block of level l if all four are valid, else 0."""
    out = [np.asarray(depth, np.float64)]
    for _ in range(1, levels):
        d = out[-1]
        h, w = d.shape[0] // 2, d.shape[1] // 2
        b = d[:2 * h, :2 * w].reshape(h, 2, w, 2)
        ok = (b > 0).all(axis=(1, 3))
        out.append(np.where(ok, b.mean(axis=(1, 3)), 0.0))
    return out


def vertex_normal_map(depth: np.ndarray, cam, depth_scale: float = 1.0):
    """Camera-frame points (eq. reprojection) and cross-product normals facing the camera.

    Returns V (H,W,3), N (H,W,3), valid-normal mask (H,W)."""
    z = np.asarray(depth, np.float64) * depth_scale
    H, W = z.shape
    vv, uu = np.mgrid[0:H, 0:W].astype(np.float64)
    V = np.stack([z * (uu - cam.cx) / cam.fx, z * (vv - cam.cy) / cam.fy, z], axis=-1)
    pv = z > 0
    N = np.zeros_like(V)
    ok = np.zeros_like(pv)
    dx = V[1:-1, 2:] - V[1:-1, :-2]
    dy = V[2:, 1:-1] - V[:-2, 1:-1]
    n = np.cross(dx, dy)
    ln = np.linalg.norm(n, axis=-1)
    inner = pv[1:-1, 1:-1] & pv[1:-1, 2:] & pv[1:-1, :-2] & pv[2:, 1:-1] & pv[:-2, 1:-1] & (ln > 0)
    n = n / np.where(ln > 0, ln, 1.0)[..., None]
    flip = (n * V[1:-1, 1:-1]).sum(-1) > 0
    n = np.where(flip[..., None], -n, n)
    N[1:-1, 1:-1] = np.where(inner[..., None], n, 0.0)
    ok[1:-1, 1:-1] = inner
    return V, N, ok


def _shifted(A: np.ndarray, du: int, dv: int) -> np.ndarray:
    """A[v + dv, u + du] with zeros outside the image."""
    H, W = A.shape[:2]
    out = np.zeros_like(A)
    ys, yd = (slice(dv, H), slice(0, H - dv)) if dv >= 0 else (slice(0, H + dv), slice(-dv, H))
    xs, xd = (slice(du, W), slice(0, W - du)) if du >= 0 else (slice(0, W + du), slice(-du, W))
    out[yd, xd] = A[ys, xs]
    return out


def depth_support_filter(depth: np.ndarray, support_rel: float = 0.02,
                         min_support: int = 2) -> np.ndarray:
    """Depth outlier filter (Sec. 7): a pixel keeps its depth only if at least ``min_support``
    of its eight neighbours hold a depth that supports it, |D(q) - D(p)| <= support_rel D(p);
    discarded pixels become 0."""
    D = np.asarray(depth, np.float64)
    cnt = np.zeros(D.shape, np.int64)
    for dv in (-1, 0, 1):
        for du in (-1, 0, 1):
            if du == 0 and dv == 0:
                continue
            Q = _shifted(D, du, dv)
            cnt += (Q > 0) & (np.abs(Q - D) <= support_rel * D)
    return np.where((D > 0) & (cnt >= min_support), D, 0.0)


def bilateral_depth(depth: np.ndarray, sigma_d: float = 5.0, sigma_r: float = 0.025,
                    radius: int = 5) -> np.ndarray:
    """Bilateral depth filter (Sec. 8 parameters; Tomasi and Manduchi's definition): the
    weighted mean over the valid pixels q of the (2 radius + 1)^2 window of p with weights
    exp(-|q - p|^2 / (2 sigma_d^2)) exp(-(D(q) - D(p))^2 / (2 sigma_r^2)); invalid pixels
    (depth 0) stay 0 and contribute nothing."""
    D = np.asarray(depth, np.float64)
    num = np.zeros_like(D)
    den = np.zeros_like(D)
    for dv in range(-radius, radius + 1):
        for du in range(-radius, radius + 1):
            Q = _shifted(D, du, dv)
            w = (math.exp(-(du * du + dv * dv) / (2.0 * sigma_d ** 2)) *
                 np.exp(-(Q - D) ** 2 / (2.0 * sigma_r ** 2)) * (Q > 0))
            num += w * Q
            den += w
    return np.where(D > 0, num / np.where(den > 0, den, 1.0), 0.0)


def bilateral_normal(N: np.ndarray, sigma_d: float = 2.5, sigma_r_deg: float = 5.0,
                     radius: int = 5) -> np.ndarray:
    """Bilateral normal filter (Sec. 7, Sec. 8 parameters): the normalised weighted sum of
    the valid normals of the window with weights exp(-|q - p|^2 / (2 sigma_d^2))
    exp(-angle(n_q, n_p)^2 / (2 sigma_r^2)), the angle in degrees; pixels without a normal
    (all zero) stay zero and contribute nothing."""
    N = np.asarray(N, np.float64)
    valid = np.any(N != 0, axis=-1)
    acc = np.zeros_like(N)
    for dv in range(-radius, radius + 1):
        for du in range(-radius, radius + 1):
            Q = _shifted(N, du, dv)
            qv = _shifted(valid, du, dv)
            c = np.clip((N * Q).sum(-1), -1.0, 1.0)
            ang = np.degrees(np.arccos(c))
            w = (math.exp(-(du * du + dv * dv) / (2.0 * sigma_d ** 2)) *
                 np.exp(-ang ** 2 / (2.0 * sigma_r_deg ** 2)) * qv)
            acc += w[..., None] * Q
    ln = np.linalg.norm(acc, axis=-1)
    return np.where((valid & (ln > 0))[..., None], acc / np.where(ln > 0, ln, 1.0)[..., None],
                    0.0)


@dataclasses.dataclass
class Preprocess:
    """Live-frame preprocessing of the registration (Sec. 7, Sec. 8 parameters): the support
    and bilateral depth filters before the pyramid, the bilateral normal filter on every
    level's normals (normal_radius 0: none)."""
    support_rel: float = f32(0.02)
    min_support: int = 2
    sigma_d: float = 5.0
    sigma_r: float = f32(0.025)
    radius: int = 5
    normal_sigma_d: float = 2.5
    normal_sigma_r_deg: float = 5.0
    normal_radius: int = 5

    def depth(self, depth: np.ndarray) -> np.ndarray:
        D = np.asarray(depth, np.float64)
        if self.min_support > 0:
            D = depth_support_filter(D, self.support_rel, self.min_support)
        if self.radius > 0:
            D = bilateral_depth(D, self.sigma_d, self.sigma_r, self.radius)
        return D

    def normals(self, N: np.ndarray) -> np.ndarray:
        if self.normal_radius <= 0:
            return N
        return bilateral_normal(N, self.normal_sigma_d, self.normal_sigma_r_deg,
                                self.normal_radius)


def post_fusion_mae(rendered: np.ndarray, measured: np.ndarray):
    """Geometric post-fusion error (Sec. 8): the mean absolute difference between the depth
    rendered at a pose after fusion and the input depth of that pose, over the pixels where
    both are valid.  Returns (mean, pixel count)."""
    r = np.asarray(rendered, np.float64)
    m = np.asarray(measured, np.float64)
    both = (r > 0) & (m > 0)
    n = int(both.sum())
    return (float(np.abs(r - m)[both].sum() / n) if n else 0.0), n


@dataclasses.dataclass
class IcpParams:
    dist: float = 0.10                     # reject ||q - y|| above this [m]
    angle_deg: float = 20.0                # reject normal angle above this
    weight: str = "const"                  # "const" or "icp" (eq. ICP_weight)
    z_min: float = 0.1


def associate_reduce(live_V, live_N, live_ok, model_V, model_N, model_mask, cam_model,
                     dT: np.ndarray, dim: int, params: IcpParams = IcpParams()):
    """One Gauss-Newton linearisation around xi = 0 (Sec. 5).

    Returns H (dim x dim), g (dim), error sum, inlier count.  H = sum w J J^T and
    g = sum w J r (the factor 2 of eq. ICP_Hessian cancels in eq. ICP_solution)."""
    P = live_V[live_ok].reshape(-1, 3)
    Nl = live_N[live_ok].reshape(-1, 3)
    R, t = dT[:3, :3], dT[:3, 3]
    y = P @ R.T + t
    nl = Nl @ R.T
    # scale-aware rotation of normals: normalise after applying R (a Sim(3) dT has sR)
    nl = nl / np.linalg.norm(nl, axis=1, keepdims=True)
    pos = y[:, 2] > 0
    zz = np.where(pos, y[:, 2], 1.0)
    uf = cam_model.fx * y[:, 0] / zz + cam_model.cx
    vf = cam_model.fy * y[:, 1] / zz + cam_model.cy
    u = np.floor(uf + 0.5).astype(np.int64)
    v = np.floor(vf + 0.5).astype(np.int64)
    H_, W_ = model_mask.shape
    inb = pos & (u >= 0) & (v >= 0) & (u < W_) & (v < H_)
    u = np.where(inb, u, 0)
    v = np.where(inb, v, 0)
    has = inb & (model_mask[v, u] > 0)
    q = model_V[v, u]
    n = model_N[v, u]
    diff = q - y
    ok = has & (np.linalg.norm(diff, axis=1) <= params.dist) & \
        ((n * nl).sum(1) >= math.cos(math.radians(params.angle_deg)))
    y, n, diff = y[ok], n[ok], diff[ok]
    r = (diff * n).sum(1)
    J = np.concatenate([-n, -np.cross(y, n)], axis=1)
    if dim == 7:
        J = np.concatenate([J, -(n * y).sum(1, keepdims=True)], axis=1)
    if params.weight == "icp":
        z = P[ok][:, 2]
        w = 1.0 / (z + (1.0 - params.z_min)) ** 2           # eq. ICP_weight
    else:
        w = np.ones(len(r))
    H = (J * w[:, None]).T @ J
    g = (J * w[:, None]).T @ r
    return H, g, float((w * r * r).sum()), int(ok.sum())


# ----------------------------------------------------------------------------------------
# Photometric terms of combined ICP (Sec. 5.2, eq. combined_icp; Sec. 5.3, eq. keyframe_icp,
# eq. keyframe_icp_derivative, eq. wedge_operator, eq. projection_dx)
# ----------------------------------------------------------------------------------------

def intensity(rgb: np.ndarray) -> np.ndarray:
    """Grey value in [0, 1] of an 8-bit RGB image: (0.299 R + 0.587 G + 0.114 B) / 255."""
    c = np.asarray(rgb, np.float64)
    return (0.299 * c[..., 0] + 0.587 * c[..., 1] + 0.114 * c[..., 2]) / 255.0


def intensity_pyramid(I: np.ndarray, levels: int):
    """Level l+1 pixel = mean of its 2x2 block of level l."""
    out = [np.asarray(I, np.float64)]
    for _ in range(1, levels):
        a = out[-1]
        h, w = a.shape[0] // 2, a.shape[1] // 2
        out.append(a[:2 * h, :2 * w].reshape(h, 2, w, 2).mean(axis=(1, 3)))
    return out


def image_gradient(I: np.ndarray):
    """Central differences (I(u+1) - I(u-1)) / 2 per pixel; zero on the border pixels."""
    gx = np.zeros_like(I)
    gy = np.zeros_like(I)
    gx[:, 1:-1] = 0.5 * (I[:, 2:] - I[:, :-2])
    gy[1:-1, :] = 0.5 * (I[2:, :] - I[:-2, :])
    return gx, gy


def bilinear(I: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Bilinear interpolation at (u, v), pixel centres at integer coordinates; callers keep
    u in [0, W - 1) and v in [0, H - 1)."""
    u0 = np.floor(u).astype(np.int64)
    v0 = np.floor(v).astype(np.int64)
    a, b = u - u0, v - v0
    return ((1 - a) * (1 - b) * I[v0, u0] + a * (1 - b) * I[v0, u0 + 1] +
            (1 - a) * b * I[v0 + 1, u0] + a * b * I[v0 + 1, u0 + 1])


def photometric_terms(P: np.ndarray, I_live: np.ndarray, I_ref: np.ndarray, cam_ref,
                      T_ref_model: np.ndarray, dT: np.ndarray, dim: int, max_err: float):
    """Residuals r = I_live - I_ref(pi(K T_RS dT p)) and their Jacobians (eq. keyframe_icp).

    P (n,3): live points (live camera frame), I_live (n): their live grey values.
    The warped point a = T_RS dT p must lie in front of the reference camera and project to
    (u, v) in [1, W - 2] x [1, H - 2], so that the 2x2 interpolation stencil has central
    differences; |r| <= max_err.  The Jacobian is the derivative of r itself,
    -grad I_ref . dpi/da . R(T_RS) [I | -(dT p)^] (eq. keyframe_icp_derivative with the sign of
    the residual; the projection derivative has -x/z^2 in its first row), and for Sim(3) the
    scale column -grad I_ref . dpi/da . R(T_RS) (dT p).
    Returns (J (m, dim), r (m,), mask over the n points)."""
    y = P @ dT[:3, :3].T + dT[:3, 3]
    Rr, tr = T_ref_model[:3, :3], T_ref_model[:3, 3]
    a = y @ Rr.T + tr
    H_, W_ = I_ref.shape
    pos = a[:, 2] > 0
    z = np.where(pos, a[:, 2], 1.0)
    u = cam_ref.fx * a[:, 0] / z + cam_ref.cx
    v = cam_ref.fy * a[:, 1] / z + cam_ref.cy
    ok = pos & (u >= 1) & (u <= W_ - 2) & (v >= 1) & (v <= H_ - 2)
    u = np.where(ok, u, 1.0)
    v = np.where(ok, v, 1.0)
    gx_img, gy_img = image_gradient(I_ref)
    Ik = bilinear(I_ref, u, v)
    gx = bilinear(gx_img, u, v)
    gy = bilinear(gy_img, u, v)
    r = I_live - Ik
    ok &= np.abs(r) <= max_err
    # d pixel / d a
    du = np.stack([cam_ref.fx / z, np.zeros_like(z), -cam_ref.fx * a[:, 0] / z ** 2], 1)
    dv = np.stack([np.zeros_like(z), cam_ref.fy / z, -cam_ref.fy * a[:, 1] / z ** 2], 1)
    dI_da = gx[:, None] * du + gy[:, None] * dv          # (n, 3)
    dI_dy = dI_da @ Rr                                    # row vectors: dI/da R
    J = np.concatenate([-dI_dy, -np.cross(y, dI_dy)], 1)  # -dI/dy [I | -y^]
    if dim == 7:
        J = np.concatenate([J, -(dI_dy * y).sum(1, keepdims=True)], 1)
    return J[ok], r[ok], ok


def associate_reduce_rgb(live_V, live_N, live_ok, live_I, model_V, model_N, model_mask,
                         cam_model, I_ref, cam_ref, T_ref_model, dT, dim,
                         params: IcpParams = IcpParams(), lam: float = 0.1,
                         max_err: float = 0.05):
    """Normal equations of combined ICP (eq. combined_icp): the geometric sums of
    associate_reduce plus lam times the photometric sums over every live pixel with depth;
    both terms carry the live pixel's depth weight (Sec. 5.2)."""
    H, g, err, cnt = associate_reduce(live_V, live_N, live_ok, model_V, model_N, model_mask,
                                      cam_model, dT, dim, params)
    has = live_V[..., 2] > 0
    P = live_V[has].reshape(-1, 3)
    Jp, rp, okp = photometric_terms(P, np.asarray(live_I)[has], I_ref, cam_ref, T_ref_model,
                                    dT, dim, max_err)
    if params.weight == "icp":
        z = P[okp][:, 2]
        w = 1.0 / (z + (1.0 - params.z_min)) ** 2
    else:
        w = np.ones(len(rp))
    H = H + lam * (Jp * w[:, None]).T @ Jp
    g = g + lam * (Jp * w[:, None]).T @ rp
    err = err + lam * float((w * rp * rp).sum())
    return H, g, err, cnt, int(okp.sum())


def solve_step(H: np.ndarray, g: np.ndarray) -> np.ndarray:
    """xi = -H^{-1} g via Cholesky (eq. ICP_solution)."""
    c = scipy.linalg.cho_factor(H, lower=True)
    return -scipy.linalg.cho_solve(c, g)


# ----------------------------------------------------------------------------------------
# Levenberg-Marquardt with Madsen's damping (Sec. 7) and scale anchoring (Sec. 6)
# ----------------------------------------------------------------------------------------

@dataclasses.dataclass
class LmState:
    """Damping state of one Levenberg-Marquardt run (Madsen, Nielsen and Tingleff 2004):
    mu, nu and the accepted iterate's normal equations H, g and error F = sum w r^2."""
    tau: float = 1e-3
    mu: float = 0.0
    nu: float = 2.0
    started: bool = False
    H: Optional[np.ndarray] = None
    g: Optional[np.ndarray] = None
    F: float = 0.0
    h: Optional[np.ndarray] = None       # last step, taken from the accepted iterate


def lm_update(st: LmState, H: np.ndarray, g: np.ndarray, F: float) -> bool:
    """Takes the normal equations (H = sum w J J^T, g = sum w J r, F = sum w r^2) at the
    candidate iterate; returns True if the candidate is accepted.  The first call accepts and
    sets mu = tau max(diag H).  Later calls compute the gain ratio
    rho = (F_acc - F) / (h^T (mu h - g_acc)) of the last step h (the ratio of actual to
    predicted reduction of the cost 1/2 sum w r^2); rho > 0 accepts the candidate and scales
    mu by max(1/3, 1 - (2 rho - 1)^3) with nu = 2, otherwise mu *= nu and nu *= 2."""
    if not st.started:
        st.started = True
        st.mu = st.tau * float(np.max(np.diag(H)))
        st.nu = 2.0
        st.H, st.g, st.F = H, g, F
        return True
    h = st.h
    pred = float(h @ (st.mu * h - st.g))
    rho = (st.F - F) / pred if pred > 0 else -1.0
    if rho > 0:
        st.mu *= max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
        st.nu = 2.0
        st.H, st.g, st.F = H, g, F
        return True
    st.mu *= st.nu
    st.nu *= 2.0
    return False


def lm_step(st: LmState) -> np.ndarray:
    """The next step from the accepted iterate: (H + mu I) h = -g (Cholesky)."""
    A = st.H + st.mu * np.eye(st.H.shape[0])
    st.h = solve_step(A, st.g)
    return st.h


def icp_lm(live_depth: np.ndarray, live_cam, model_levels, dT0: np.ndarray, dim: int = 7,
           iters=(10, 5, 4), params: IcpParams = IcpParams(), tau: float = 1e-3,
           min_step: float = 1e-6, depth_scale: float = 1.0, min_inliers_per_dim: int = 64):
    """Coarse-to-fine point-to-plane ICP solved by Levenberg-Marquardt with Madsen's damping
    (Sec. 7); the damping restarts at every level.  Each iteration associates and reduces at
    the candidate pose, accepts or rejects it, and steps from the accepted pose; the result
    is the last accepted pose.  With tau = 0 it is the Gauss-Newton iteration of icp()."""
    L = len(model_levels)
    pyr = depth_pyramid(live_depth, L)
    dT = np.array(dT0, np.float64)
    log = []
    for l in reversed(range(L)):
        V, N, ok = vertex_normal_map(pyr[l], live_cam.level(l), depth_scale)
        mV, mN, mM, mcam = model_levels[l]
        st = LmState(tau=tau)
        cand = dT.copy()
        for _ in range(iters[l]):
            H, g, err, cnt = associate_reduce(V, N, ok, mV, mN, mM, mcam, cand, dim, params)
            if cnt < min_inliers_per_dim * dim:
                log.append(dict(level=l, status="degenerate", inliers=cnt))
                break
            acc = lm_update(st, H, g, err)
            if acc:
                dT = cand
            h = lm_step(st)
            cand = exp_map(h) @ dT
            log.append(dict(level=l, inliers=cnt, err=err, accepted=acc, mu=st.mu,
                            step=float(np.linalg.norm(h))))
            if np.linalg.norm(h) < min_step:
                break
    return dT, log


def anchored_log_scales(log_scales: Sequence[float], anchor: float) -> np.ndarray:
    """Scale anchoring (Sec. 6, eq. scale_anchor, read as a difference of log scales): the
    compensated log scale of each sensor is its estimate minus the anchor sensor's."""
    return np.asarray(log_scales, np.float64) - float(anchor)


def icp_rgb(live_depth: np.ndarray, live_rgb: np.ndarray, live_cam, model_levels,
            ref_levels, T_ref_model: np.ndarray, dT0: np.ndarray, dim: int = 6,
            iters=(10, 5, 4), params: IcpParams = IcpParams(), lam: float = 0.1,
            max_err=(0.05, 0.175, 0.175), min_step: float = 1e-6, depth_scale: float = 1.0,
            min_inliers_per_dim: int = 64):
    """Coarse-to-fine combined geometric + photometric ICP (Sec. 5.2, Sec. 5.3).

    ref_levels[l] = (I_ref, cam_ref) is the reference grey image at level l (a keyframe, the
    previous frame or a rendered colour image), T_ref_model maps the model camera frame to
    the reference camera frame (identity for frame-to-frame and frame-to-render).  The live
    grey pyramid halves by 2x2 means.  max_err[l] is the intensity outlier threshold of
    level l (fine 0.05, coarse 0.175)."""
    L = len(model_levels)
    pyr = depth_pyramid(live_depth, L)
    ipyr = intensity_pyramid(intensity(live_rgb), L)
    dT = np.array(dT0, np.float64)
    log = []
    for l in reversed(range(L)):
        V, N, ok = vertex_normal_map(pyr[l], live_cam.level(l), depth_scale)
        mV, mN, mM, mcam = model_levels[l]
        I_ref, rcam = ref_levels[l]
        for _ in range(iters[l]):
            H, g, err, cnt, cph = associate_reduce_rgb(V, N, ok, ipyr[l], mV, mN, mM, mcam,
                                                       I_ref, rcam, T_ref_model, dT, dim,
                                                       params, lam, max_err[l])
            if cnt < min_inliers_per_dim * dim:
                log.append(dict(level=l, status="degenerate", inliers=cnt))
                break
            xi = solve_step(H, g)
            dT = exp_map(xi) @ dT
            log.append(dict(level=l, inliers=cnt, photometric=cph, err=err,
                            step=float(np.linalg.norm(xi)), xi=xi))
            if np.linalg.norm(xi) < min_step:
                break
    return dT, log


def icp(live_depth: np.ndarray, live_cam, model_levels, dT0: np.ndarray, dim: int = 6,
        iters=(10, 5, 4), params: IcpParams = IcpParams(), min_step: float = 1e-6,
        depth_scale: float = 1.0, min_inliers_per_dim: int = 64,
        preprocess: Optional[Preprocess] = None):
    """Coarse-to-fine point-to-plane ICP.

    model_levels[l] = (V, N, mask, cam) rendered at level l (model camera frame).
    ``iters`` lists fine-to-coarse iteration counts; levels run coarse to fine.
    ``preprocess`` filters the live depth before the pyramid and every level's normals.
    Returns the final live->model transform and a per-iteration log."""
    L = len(model_levels)
    if preprocess is not None:
        live_depth = preprocess.depth(live_depth)
    pyr = depth_pyramid(live_depth, L)
    dT = np.array(dT0, np.float64)
    log = []
    for l in reversed(range(L)):
        V, N, ok = vertex_normal_map(pyr[l], live_cam.level(l), depth_scale)
        if preprocess is not None:
            N = preprocess.normals(N)
        mV, mN, mM, mcam = model_levels[l]
        for _ in range(iters[l]):
            H, g, err, cnt = associate_reduce(V, N, ok, mV, mN, mM, mcam, dT, dim, params)
            if cnt < min_inliers_per_dim * dim:
                log.append(dict(level=l, status="degenerate", inliers=cnt))
                break
            xi = solve_step(H, g)
            dT = exp_map(xi) @ dT                              # eq. deltaT_update
            log.append(dict(level=l, inliers=cnt, err=err, step=float(np.linalg.norm(xi)),
                            xi=xi))
            if np.linalg.norm(xi) < min_step:
                break
    return dT, log
