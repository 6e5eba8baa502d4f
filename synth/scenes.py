"""Analytic scenes, camera poses and RGB-D frames with seeded noise.

Conventions (shared with every consumer):

* Units are metres.  Cameras use the pinhole model with OpenCV axes (x right, y down,
  z forward).  A pose ``T_wc`` is a 4x4 float64 matrix mapping camera to world coordinates.
* Pixel (u, v) has its centre at integer coordinates; the ray of pixel (u, v) passes through
  camera point ((u - cx) / fx, (v - cy) / fy, 1).
* A depth image holds the camera-frame z of the first surface along the pixel ray, float32,
  with 0 marking "no measurement".  Colour images are HxWx3 uint8.

The workloads follow the paper's RGB-D setting (depth cameras, 5 mm to 4 cm voxels,
Kinect-like noise growing with depth as discussed in Sec. 5.1) with seeded analytic scenes
standing in for the public datasets of Sec. 8, which are not used.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch


# ----------------------------------------------------------------------------------------
# Cameras and poses
# ----------------------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    def level(self, l: int) -> "Camera":
        """Intrinsics of pyramid level ``l`` (each level halves the resolution).

        Pixel centres map as c_l = (c + 0.5) / 2^l - 0.5 so that a 2x2 block of fine pixels
        averages onto one coarse pixel centred on their mean position."""
        if l == 0:
            return self
        s = 2.0 ** l
        return Camera(self.width >> l, self.height >> l, self.fx / s, self.fy / s,
                      (self.cx + 0.5) / s - 0.5, (self.cy + 0.5) / s - 0.5)

    def pixel_rays(self) -> np.ndarray:
        """Unnormalised camera-frame ray (x, y, 1) per pixel, shape (H, W, 3), float64."""
        u = np.arange(self.width, dtype=np.float64)
        v = np.arange(self.height, dtype=np.float64)
        uu, vv = np.meshgrid(u, v)
        return np.stack([(uu - self.cx) / self.fx, (vv - self.cy) / self.fy,
                         np.ones_like(uu)], axis=-1)


def look_at(eye: Sequence[float], target: Sequence[float],
            up: Sequence[float] = (0.0, 0.0, 1.0)) -> np.ndarray:
    """Camera-to-world pose of a camera at ``eye`` whose optical axis points at ``target``."""
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    x = np.cross(z, np.asarray(up, np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    T = np.eye(4)
    T[:3, 0], T[:3, 1], T[:3, 2], T[:3, 3] = x, y, z, eye
    return T


def random_rotation_small(axis: np.ndarray, angle: float) -> np.ndarray:
    """Rotation matrix of ``angle`` radians about unit ``axis`` (Rodrigues' formula)."""
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1.0 - math.cos(angle)) * (K @ K)


def _unit(rng: np.random.Generator) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def perturb_pose(trans: float, angle: float, rng: np.random.Generator) -> np.ndarray:
    """A rigid 4x4 offset: rotation by ``angle`` about a random axis and a translation of
    length ``trans`` along another random axis."""
    D = np.eye(4)
    D[:3, :3] = random_rotation_small(_unit(rng), angle)
    D[:3, 3] = trans * _unit(rng)
    return D


# ----------------------------------------------------------------------------------------
# Primitives and ray intersection
# ----------------------------------------------------------------------------------------

@dataclasses.dataclass
class Sphere:
    center: np.ndarray
    radius: float
    albedo: np.ndarray          # (3,) uint8


@dataclasses.dataclass
class Box:
    """Solid axis-aligned box; ``face_albedo`` (6,3) colours the faces -x,+x,-y,+y,-z,+z."""
    lo: np.ndarray
    hi: np.ndarray
    face_albedo: np.ndarray     # (6, 3) uint8


@dataclasses.dataclass
class Room:
    """Hollow axis-aligned room seen from inside; walls face inwards."""
    lo: np.ndarray
    hi: np.ndarray
    face_albedo: np.ndarray     # (6, 3) uint8, walls at -x,+x,-y,+y,-z,+z


@dataclasses.dataclass
class Scene:
    spheres: List[Sphere]
    boxes: List[Box]
    room: Optional[Room] = None


def _hit_sphere(o, d, s: Sphere):
    c = torch.as_tensor(s.center, dtype=d.dtype, device=d.device)
    oc = o - c
    b = d @ oc
    cc = oc @ oc - s.radius ** 2
    disc = b * b - cc
    ok = disc >= 0
    sq = torch.sqrt(torch.clamp(disc, min=0.0))
    t0 = -b - sq
    t1 = -b + sq
    inf = torch.full_like(b, math.inf)
    t = torch.where(t0 > 1e-9, t0, torch.where(t1 > 1e-9, t1, inf))
    t = torch.where(ok, t, inf)
    p = o + d * torch.where(torch.isfinite(t), t, torch.zeros_like(t))[:, None]
    n = (p - c) / s.radius
    alb = torch.as_tensor(s.albedo, device=d.device).expand(d.shape[0], 3)
    return t, n, alb


def _slabs(o, d, lo, hi):
    lo = torch.as_tensor(lo, dtype=d.dtype, device=d.device)
    hi = torch.as_tensor(hi, dtype=d.dtype, device=d.device)
    par = d == 0
    dd = torch.where(par, torch.ones_like(d), d)
    t1 = (lo - o) / dd
    t2 = (hi - o) / dd
    tmin = torch.minimum(t1, t2)
    tmax = torch.maximum(t1, t2)
    # rays parallel to a slab: inside -> (-inf, inf), outside -> empty
    inside = ((o >= lo) & (o <= hi)).expand_as(d)
    ninf = torch.full_like(d, -math.inf)
    pinf = torch.full_like(d, math.inf)
    tmin = torch.where(par, torch.where(inside, ninf, pinf), tmin)
    tmax = torch.where(par, torch.where(inside, pinf, ninf), tmax)
    return tmin, tmax


def _face_normal(d, ax, sign):
    n = torch.zeros_like(d)
    n.scatter_(1, ax[:, None], sign[:, None])
    return n


def _hit_box(o, d, b: Box):
    tmin, tmax = _slabs(o, d, b.lo, b.hi)
    t_enter, ax = tmin.max(dim=1)
    t_exit = tmax.min(dim=1).values
    ok = (t_enter <= t_exit) & (t_enter > 1e-9)
    t = torch.where(ok, t_enter, torch.full_like(t_enter, math.inf))
    sign = -torch.sign(d.gather(1, ax[:, None])[:, 0])   # outward normal faces the ray
    face = 2 * ax + (sign > 0).long()
    alb = torch.as_tensor(b.face_albedo, device=d.device)[face]
    return t, _face_normal(d, ax, sign), alb


def _hit_room(o, d, r: Room):
    tmin, tmax = _slabs(o, d, r.lo, r.hi)
    t_exit, ax = tmax.min(dim=1)
    ok = t_exit > 1e-9
    t = torch.where(ok, t_exit, torch.full_like(t_exit, math.inf))
    dsign = torch.sign(d.gather(1, ax[:, None])[:, 0])
    face = 2 * ax + (dsign > 0).long()
    alb = torch.as_tensor(r.face_albedo, device=d.device)[face]
    return t, _face_normal(d, ax, -dsign), alb                # inward-facing wall


def raycast_scene(scene: Scene, origin, dirs, device: str = "cpu"):
    """First intersection of unit rays ``origin + t * dirs`` with the scene (float64).

    Returns numpy (t, normal, albedo, hit) with t = inf where nothing is hit; normals face
    the ray.  ``device`` selects where the intersection arithmetic runs (torch).
    """
    o = torch.as_tensor(np.asarray(origin, np.float64), device=device)
    d = torch.as_tensor(np.asarray(dirs, np.float64), device=device)
    n_rays = d.shape[0]
    t_best = torch.full((n_rays,), math.inf, dtype=torch.float64, device=device)
    n_best = torch.zeros((n_rays, 3), dtype=torch.float64, device=device)
    a_best = torch.zeros((n_rays, 3), dtype=torch.uint8, device=device)
    prims = [(_hit_sphere, s) for s in scene.spheres] + [(_hit_box, b) for b in scene.boxes]
    if scene.room is not None:
        prims.append((_hit_room, scene.room))
    for fn, prim in prims:
        t, n, a = fn(o, d, prim)
        closer = t < t_best
        t_best = torch.where(closer, t, t_best)
        n_best = torch.where(closer[:, None], n, n_best)
        a_best = torch.where(closer[:, None], a, a_best)
    hit = torch.isfinite(t_best)
    return (t_best.cpu().numpy(), n_best.cpu().numpy(), a_best.cpu().numpy(),
            hit.cpu().numpy())


def solid_texture(points: np.ndarray, period: float) -> np.ndarray:
    """Smooth brightness factor in [0.2, 1.0] of world points (n, 3): a solid texture, the same
    from every view, so that photometric registration has image gradients to work with."""
    k = 2.0 * math.pi / period
    x, y, z = points[:, 0], points[:, 1], points[:, 2]
    return 0.6 + 0.25 * np.sin(k * x) * np.cos(k * y) + 0.15 * np.sin(k * z + 1.3)


def render_frame(scene: Scene, cam: Camera, T_wc: np.ndarray, *, noise: str = "none",
                 sigma: float = 0.0, seed: Optional[int] = None, z_max: float = 10.0,
                 depth_scale: float = 1.0, device: str = "cpu",
                 texture_period: Optional[float] = None):
    """Analytic RGB-D frame.

    noise: "none", "const" (N(0, sigma^2)) or "quadratic" (N(0, (sigma * z^2)^2)); the
    noise is drawn with numpy from ``seed`` so every device sees identical frames.
    ``depth_scale`` multiplies every stored depth (a sensor with a wrong depth scale).
    ``texture_period`` (metres) modulates every albedo by ``solid_texture`` of the hit
    point.
    Returns dict with depth (H,W float32), rgb (H,W,3 uint8), true depth (float64),
    camera-frame unit normals (H,W,3 float64, facing the camera) and hit mask.
    """
    rays = cam.pixel_rays().reshape(-1, 3)
    norm = np.linalg.norm(rays, axis=1)
    d_cam = rays / norm[:, None]
    R = T_wc[:3, :3]
    d_w = d_cam @ R.T
    t, n_w, alb, hit = raycast_scene(scene, T_wc[:3, 3], d_w, device=device)
    z = np.where(hit, t / norm, 0.0)
    hit &= (z <= z_max) & (z > 0)
    z = np.where(hit, z, 0.0)
    zn = z.copy()
    if noise != "none":
        rng = np.random.default_rng(seed)
        e = rng.normal(size=z.shape)
        if noise == "const":
            zn = z + sigma * e
        elif noise == "quadratic":
            zn = z + sigma * z * z * e
        else:
            raise ValueError(noise)
        zn = np.where(hit & (zn > 0), zn, 0.0)
    depth = (zn * depth_scale).astype(np.float32).reshape(cam.height, cam.width)
    if texture_period is not None:
        pts = T_wc[:3, 3] + d_w * np.where(hit, t, 0.0)[:, None]
        alb = np.clip(np.rint(alb * solid_texture(pts, texture_period)[:, None]), 0, 255)
    rgb = np.where(hit[:, None], alb, 0).astype(np.uint8).reshape(cam.height, cam.width, 3)
    n_c = n_w @ R            # world -> camera: R^T n, written row-wise
    return dict(depth=depth, rgb=rgb, true_depth=z.reshape(cam.height, cam.width),
                normal=n_c.reshape(cam.height, cam.width, 3),
                hit=hit.reshape(cam.height, cam.width))


# ----------------------------------------------------------------------------------------
# Tiny scene: sphere r = 0.2 m at the origin plus a 1 cm plate at x = 0.3 m
# ----------------------------------------------------------------------------------------

TINY_CAMERA = Camera(160, 120, 120.0, 120.0, 80.0, 60.0)
TINY_PLATE_FRONT = np.array([40, 200, 60], np.uint8)     # +x face
TINY_PLATE_BACK = np.array([200, 40, 160], np.uint8)     # -x face


def tiny_scene() -> Scene:
    plate_alb = np.tile(np.array([120, 120, 120], np.uint8), (6, 1))
    plate_alb[0] = TINY_PLATE_BACK
    plate_alb[1] = TINY_PLATE_FRONT
    return Scene(
        spheres=[Sphere(np.zeros(3), 0.2, np.array([210, 90, 50], np.uint8))],
        boxes=[Box(np.array([0.295, -0.30, -0.30]), np.array([0.305, 0.30, 0.30]), plate_alb)],
    )


def tiny_cameras(n: int = 10, seed: int = 1) -> List[np.ndarray]:
    """Poses on the radius-1 m circle in the world z = 0 plane looking at the origin."""
    rng = np.random.default_rng(seed)
    phis = rng.uniform(0.0, 2.0 * math.pi, n)
    return [look_at((math.cos(p), math.sin(p), 0.0), (0, 0, 0)) for p in phis]


def tiny_render_pose(phi: float = 0.3) -> np.ndarray:
    return look_at((math.cos(phi), math.sin(phi), 0.0), (0, 0, 0))


def tiny_frames(n: int = 10, sigma: float = 0.0005, cam: Camera = TINY_CAMERA):
    """The tiny workload: ``n`` noisy frames (seed 1000 + k for frame k) and their poses."""
    sc = tiny_scene()
    out = []
    for k, T in enumerate(tiny_cameras(n)):
        f = render_frame(sc, cam, T, noise="const" if sigma > 0 else "none", sigma=sigma,
                         seed=1000 + k, z_max=10.0)
        f["T_wc"] = T
        out.append(f)
    return out


# Dense block range of the tiny map: blocks x -3..4, y and z -4..3 (8^3 blocks of 8^3 voxels).
TINY_DENSE_LO = (-3, -4, -4)
TINY_DENSE_HI = (4, 3, 3)


# ----------------------------------------------------------------------------------------
# Room scene: 4 x 4 x 3 m room with seeded boxes, spheres and 5 mm plates
# ----------------------------------------------------------------------------------------

ROOM_CAMERA = Camera(640, 480, 525.0, 525.0, 319.5, 239.5)


def room_pose(k: int, n: int = 300) -> np.ndarray:
    t = k / n
    c = (2.0 + math.cos(2 * math.pi * t), 2.0 + 0.8 * math.sin(2 * math.pi * t),
         1.5 + 0.2 * math.sin(4 * math.pi * t))
    tgt = (2.0 - 0.8 * math.cos(2 * math.pi * t), 2.0 - 0.8 * math.sin(2 * math.pi * t), 1.0)
    return look_at(c, tgt)


def _path_points(n: int = 600) -> np.ndarray:
    return np.array([room_pose(k, n)[:3, 3] for k in range(n)])


def room_scene(seed: int = 7, n_boxes: int = 8, n_spheres: int = 6, n_plates: int = 6,
               tube: float = 0.6) -> Scene:
    rng = np.random.default_rng(seed)
    path = _path_points()
    lo_b = np.array([0.3, 0.3, 0.0])
    hi_b = np.array([3.7, 3.7, 2.5])

    def clear(lo, hi) -> bool:
        # distance from the path to the AABB must exceed the tube radius
        q = np.clip(path, lo, hi)
        return bool(np.min(np.linalg.norm(path - q, axis=1)) > tube)

    def col() -> np.ndarray:
        return rng.integers(0, 256, size=3).astype(np.uint8)

    boxes: List[Box] = []
    spheres: List[Sphere] = []
    tries = 0
    while len(boxes) < n_boxes and tries < 10000:
        tries += 1
        size = rng.uniform(0.2, 0.8, 3)
        lo = rng.uniform(lo_b, hi_b - size)
        lo[2] = 0.0 if rng.uniform() < 0.7 else lo[2]          # most boxes rest on the floor
        hi = lo + size
        if clear(lo, hi):
            boxes.append(Box(lo, hi, np.tile(col(), (6, 1))))
    tries = 0
    while len(spheres) < n_spheres and tries < 10000:
        tries += 1
        r = rng.uniform(0.1, 0.4)
        c = rng.uniform(lo_b + r, hi_b - r)
        if clear(c - r, c + r):
            spheres.append(Sphere(c, r, col()))
    tries = 0
    n_pl = 0
    while n_pl < n_plates and tries < 10000:
        tries += 1
        ax = int(rng.integers(0, 3))
        ext = rng.uniform(0.3, 1.0, 3)
        ext[ax] = 0.005
        lo = rng.uniform(lo_b, hi_b - ext)
        hi = lo + ext
        if clear(lo, hi):
            boxes.append(Box(lo, hi, np.stack([col() for _ in range(6)])))
            n_pl += 1
    walls = np.stack([col() for _ in range(6)])
    return Scene(spheres=spheres, boxes=boxes,
                 room=Room(np.zeros(3), np.array([4.0, 4.0, 3.0]), walls))


def room_camera() -> Camera:
    return ROOM_CAMERA


def room_frames(indices: Sequence[int], n: int = 300, scene: Optional[Scene] = None,
                noise: bool = True, device: str = "cpu"):
    """Frames ``indices`` of the room trajectory; depth noise N(0, (0.0012 z^2)^2), seed 2000+k."""
    sc = scene if scene is not None else room_scene()
    out = []
    for k in indices:
        T = room_pose(k, n)
        f = render_frame(sc, ROOM_CAMERA, T, noise="quadratic" if noise else "none",
                         sigma=0.0012, seed=2000 + k, z_max=10.0, device=device)
        f["T_wc"] = T
        f["index"] = k
        out.append(f)
    return out


# ----------------------------------------------------------------------------------------
# Tracking, precision and serving workloads
# ----------------------------------------------------------------------------------------

def tracking_cases(n: int = 30, seed: int = 3, trans: float = 0.02,
                   angle: float = math.radians(2.0)) -> List[Tuple[np.ndarray, np.ndarray]]:
    """(true pose on the tiny-scene circle, initial live->model offset) pairs."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        phi = rng.uniform(0.0, 2.0 * math.pi)
        T = look_at((math.cos(phi), math.sin(phi), 0.0), (0, 0, 0))
        out.append((T, perturb_pose(trans, angle, rng)))
    return out


def precision_scale(seed: int = 11) -> float:
    """Depth scale factor of the second sensor of the scaled-sensor registration workload."""
    return float(np.random.default_rng(seed).uniform(0.9, 1.1))


def serving_sensors(seed: int = 13):
    """Four simulated sensors: (Camera, depth scale factor)."""
    rng = np.random.default_rng(seed)
    out = []
    for (w, h) in [(320, 240), (640, 480), (848, 480), (1280, 720)]:
        f = rng.uniform(0.9, 1.1) * 525.0 * w / 640.0
        out.append((Camera(w, h, f, f, (w - 1) / 2.0, (h - 1) / 2.0),
                    float(rng.uniform(0.9, 1.1))))
    return out


def serving_requests(n: int = 3600, rate: float = 120.0, n_sensors: int = 4, seed: int = 14):
    """Poisson arrivals: list of (arrival time s, sensor index, circle angle, prior offset)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    sensor = rng.integers(0, n_sensors, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    offs = [perturb_pose(0.02, math.radians(2.0), rng) for _ in range(n)]
    return [(float(t[i]), int(sensor[i]), float(phi[i]), offs[i]) for i in range(n)]


def serving_workload(n: int = 240, rate: float = 120.0, seed: int = 14, sensors=None,
                     device: str = "cpu", prior_scale_error: float = 0.01):
    """Request stream of the serving workload on the tiny scene: per request the arrival
    time, the sensor index, the camera pose the model is rendered at, the live depth frame
    of that sensor at that pose (its depth scaled by the sensor's factor s, noise
    N(0, 0.5 mm^2) seeded by the request index) and the initial live -> model transform: a
    2 cm / 2 degree rigid offset whose linear part is multiplied by (1 + prior_scale_error) / s,
    i.e. a scale prior that is off by ``prior_scale_error``."""
    sensors = sensors if sensors is not None else serving_sensors()
    sc = tiny_scene()
    out = []
    for k, (t, si, phi, off) in enumerate(serving_requests(n, rate, len(sensors), seed)):
        cam, s = sensors[si]
        T = tiny_render_pose(phi)
        f = render_frame(sc, cam, T, noise="const", sigma=0.0005, seed=5000 + k,
                         depth_scale=s, device=device)
        dT0 = off.copy()
        dT0[:3, :3] *= (1.0 + prior_scale_error) / s
        out.append(dict(arrival=t, sensor=si, T_model=T, depth=f["depth"], dT0=dT0, scale=s))
    return out
