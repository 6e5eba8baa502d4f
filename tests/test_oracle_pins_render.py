"""Pins of the oracle's render branches and allocation band that the plane, sphere and plate
pins leave open (CPU only).

* Fallback branch (Sec. 4, eq. combine_tsdf_weight): a hand-built map whose defined
  directions all have zero combination weight in the gradient form -- one direction's
  normals lie beyond theta from its axis, one holds a constant (gradient-free) field, one
  faces away from the ray.  f, the root, the output normal (weighted axis vectors) and
  the colour (blended with the fallback weights) then have closed forms.
* Colour blend on the gradient branch (design reading of the output colour): two
  directions holding the same plane with different constant colours, geometric weights
  and colour weights; the blend uses w_dir(n^D) max(0, <n^D, -r>) W_c^D and not the
  geometric weights.
* Allocation band (Sec. 7, design reading of the allocation set): the blocks a frame
  requests equal, up to blocks the segment clips for less than the sample spacing, the
  blocks that an exact grid traversal of every pixel's segment p +- tau r passes through.
"""
import math

import numpy as np

from oracle import oracle as O

LOC = np.stack([np.arange(512) % 8, np.arange(512) // 8 % 8, np.arange(512) // 64], 1)


def field_blob(blocks, fields, voxel):
    """Bricks for every block in `blocks` and every direction d of `fields`
    {d: (phi(x) -> values at world points x (n, 3), W, rgb, Wc)}."""
    keys, sdf, w, rgb, wc = [], [], [], [], []
    for b in blocks:
        x = (np.asarray(b) * 8 + LOC) * voxel
        for d, (phi, W, col, Wc) in sorted(fields.items()):
            keys.append([b[0], b[1], b[2], d])
            sdf.append(phi(x))
            w.append(np.full(512, W))
            rgb.append(np.tile(np.asarray(col, np.uint8), (512, 1)))
            wc.append(np.full(512, Wc))
    return dict(keys=np.array(keys, np.int32), sdf=np.array(sdf, np.float32),
                w=np.array(w, np.float32), rgb=np.array(rgb, np.uint8),
                wc=np.array(wc, np.float32))


def blocks_around(points, voxel, margin=1):
    bmin = np.floor(points.min(0) / (8 * voxel)).astype(int) - margin
    bmax = np.floor(points.max(0) / (8 * voxel)).astype(int) + margin
    return [(i, j, k) for i in range(bmin[0], bmax[0] + 1) for j in range(bmin[1], bmax[1] + 1)
            for k in range(bmin[2], bmax[2] + 1)]


def camera_along(c, z_axis):
    """Camera-to-world pose at centre c with optical axis z_axis; a 3x3 image whose centre
    pixel (1, 1) looks along z_axis."""
    z = np.asarray(z_axis, float) / np.linalg.norm(z_axis)
    up = np.array([0.0, 0.0, 1.0]) if abs(z[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    x = np.cross(up, z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    T = np.eye(4)
    T[:3, 0], T[:3, 1], T[:3, 2], T[:3, 3] = x, y, z, c
    cam = type("Cam", (), dict(width=3, height=3, fx=100.0, fy=100.0, cx=1.0, cy=1.0))()
    return T, cam


# ---- fallback branch ---------------------------------------------------------------------

VOX, TAU = 0.01, 0.04
R_HAT = np.array([1.0, -0.5, -0.4]) / np.linalg.norm([1.0, -0.5, -0.4])
C0 = np.array([-0.3, 0.2, 0.15])
T_C = 0.5                      # the Y+ field is zero at c + T_C r
W_X, W_Y, W_Z = 3.0, 2.0, 1.5  # geometric weights
PHI_Z = 0.3                    # the constant Z+ field
COL_X, COL_Y, COL_Z = (250, 250, 250), (200, 40, 10), (40, 200, 120)


def fallback_map():
    def phi_y(x):
        return (T_C - (x - C0) @ R_HAT) / TAU          # gradient -r / tau, normal -r

    fields = {
        0: (lambda x: phi_y(x) + 0.25, W_X, COL_X, 1.0),   # X+: normals 147 deg from +x
        2: (phi_y, W_Y, COL_Y, 1.0),                       # Y+: normals 65 deg from +y
        4: (lambda x: np.full(len(x), PHI_Z), W_Z, COL_Z, 1.0),  # Z+: no gradient
    }
    seg = C0 + np.outer(np.linspace(0.15, 0.9, 16), R_HAT)
    om = O.OracleMap(O.MapParams(voxel=VOX, tau=TAU))
    om.load(field_blob(blocks_around(seg, VOX), fields, VOX))
    return om


def test_fallback_setup_has_no_gradient_weight():
    """The scene is built so that every defined direction has zero weight in the gradient
    form: w_dir is zero beyond theta = 60 degrees, and the Z+ field has no gradient."""
    p = O.MapParams(voxel=VOX, tau=TAU)
    n = -R_HAT
    assert math.degrees(math.acos(n[1])) > 60.0 and O.w_dir(p, n, 2) == 0.0
    assert math.degrees(math.acos(n[0])) > 60.0 and O.w_dir(p, n, 0) == 0.0


def test_fallback_value_closed_form():
    om = fallback_map()
    ts = np.array([0.3, 0.45, 0.5, 0.51, 0.6])
    f, d, fb = om.eval(C0 + np.outer(ts, R_HAT), R_HAT)
    assert d.all() and fb.all()
    # eq. combine_tsdf_weight: W^D max(0, <v^D, -r>); X+ faces away from the ray
    wy, wz = W_Y * max(0.0, -R_HAT[1]), W_Z * max(0.0, -R_HAT[2])
    expect = (wy * (T_C - ts) / TAU + wz * PHI_Z) / (wy + wz)
    np.testing.assert_allclose(f, expect, atol=1e-6)


def test_fallback_render_root_normal_and_colour():
    om = fallback_map()
    T, cam = camera_along(C0, R_HAT)
    r = om.render(cam, T, pixels=np.array([[1, 1]]), z_far=2.0)
    assert r.mask[0] == 1
    wy, wz = W_Y * -R_HAT[1], W_Z * -R_HAT[2]
    # f = 0 where wy (T_C - t) / tau = -wz PHI_Z
    t_star = T_C + TAU * wz * PHI_Z / wy
    assert abs(r.depth[0] - t_star) < 1e-7, (r.depth[0], t_star)   # float32 voxel values
    # output normal on the fallback branch: normalised sum of omega_D v^D (world), in the
    # camera frame
    nw = np.array([0.0, wy, wz])
    nw /= np.linalg.norm(nw)
    np.testing.assert_allclose(r.normal[0], T[:3, :3].T @ nw, atol=1e-6)
    # colour blended with the fallback weights
    col = (wy * np.array(COL_Y) + wz * np.array(COL_Z)) / (wy + wz)
    np.testing.assert_array_equal(r.rgba[0], list(np.rint(col).astype(int)) + [255])


# ---- colour blend on the gradient branch ------------------------------------------------

N45 = np.array([1.0, 1.0, 0.0]) / math.sqrt(2.0)


def test_colour_blend_uses_colour_weights():
    p0 = np.array([0.3, 0.3, 0.05])

    def plane(x):
        return (x - p0) @ N45 / TAU

    cx_, cy_, cz_ = (200, 12, 50), (20, 100, 250), (255, 255, 255)
    wcx, wcy = 3.0, 1.0
    fields = {0: (plane, 1.0, cx_, wcx),      # X+: w_dir = 1/2 at 45 degrees
              2: (plane, 4.0, cy_, wcy),      # Y+: w_dir = 1/2
              4: (plane, 2.0, cz_, 5.0)}      # Z+: w_dir = 0 (normal 90 deg from +z)
    c = p0 + 0.5 * N45
    om = O.OracleMap(O.MapParams(voxel=VOX, tau=TAU))
    om.load(field_blob(blocks_around(np.stack([p0, c]), VOX), fields, VOX))
    T, cam = camera_along(c, -N45)
    r = om.render(cam, T, pixels=np.array([[1, 1]]), z_far=2.0)
    assert r.mask[0] == 1 and abs(r.depth[0] - 0.5) < 1e-7
    np.testing.assert_allclose(r.normal[0], T[:3, :3].T @ N45, atol=1e-6)
    # w_dir(n^D) max(0, <n^D, -r>) W_c^D: equal direction factors, so the colour weights
    # decide: (3 c_x + c_y) / 4 = (155, 34, 100); the geometric weights would give
    # (c_x + 4 c_y) / 5 and equal weights (c_x + c_y) / 2
    expect = (wcx * np.array(cx_) + wcy * np.array(cy_)) / (wcx + wcy)
    np.testing.assert_array_equal(r.rgba[0], list(np.rint(expect).astype(int)) + [255])
    assert list(r.rgba[0][:3]) == [155, 34, 100]


# ---- allocation band ---------------------------------------------------------------------

def segment_blocks(a, b, block):
    """Exact traversal (Amanatides & Woo) of the segment a -> b through a grid of cubes of
    edge `block`: {block key: length of the segment inside it}."""
    d = b - a
    L = float(np.linalg.norm(d))
    cur = np.floor(a / block).astype(int)
    end = np.floor(b / block).astype(int)
    step = np.sign(d).astype(int)
    tmax, tdelta = np.full(3, np.inf), np.full(3, np.inf)
    for k in range(3):
        if d[k] != 0:
            nxt = (cur[k] + (step[k] > 0)) * block
            tmax[k] = (nxt - a[k]) / d[k]
            tdelta[k] = block / abs(d[k])
    out, t = {}, 0.0
    while True:
        tn = min(1.0, tmax.min())
        out[tuple(cur)] = out.get(tuple(cur), 0.0) + (tn - t) * L
        if tn >= 1.0 or (cur == end).all():
            if tn < 1.0:
                out[tuple(cur)] += (1.0 - tn) * L
            break
        k = int(np.argmin(tmax))
        t = tn
        cur[k] += step[k]
        tmax[k] += tdelta[k]
    return out


def test_allocation_band_equals_segment_blocks():
    vox, tau = 0.01, 0.04
    W, H, f = 40, 30, 50.0
    cam = type("Cam", (), dict(width=W, height=H, fx=f, fy=f, cx=(W - 1) / 2, cy=(H - 1) / 2))()
    # camera at the origin of a tilted frame; a plane with unit normal n_c (camera frame,
    # facing the camera) at distance 0.55 m
    ang = math.radians(17.0)
    Rz = np.array([[math.cos(ang), -math.sin(ang), 0], [math.sin(ang), math.cos(ang), 0], [0, 0, 1]])
    T = np.eye(4)
    T[:3, :3] = Rz
    T[:3, 3] = [0.013, -0.021, 0.007]
    n_c = np.array([0.2, -0.1, -1.0])
    n_c /= np.linalg.norm(n_c)
    uu, vv = np.meshgrid(np.arange(W), np.arange(H))
    rays = np.stack([(uu - cam.cx) / f, (vv - cam.cy) / f, np.ones_like(uu, float)], -1)
    t = -0.55 / (rays @ n_c)                     # <p, n_c> = -0.55 on the plane
    depth = (t * rays[..., 2]).astype(np.float32)
    om = O.OracleMap(O.MapParams(voxel=vox, tau=tau))
    keys, border, alloc = om.requests(depth, cam, T)
    requested = {tuple(k) for k, a in zip(keys, alloc) if a}
    flagged = {tuple(k) for k, b in zip(keys, border) if b}
    p = O.MapParams(voxel=vox, tau=tau)
    n_w = T[:3, :3] @ n_c
    dirs = [d for d in range(6) if O.w_dir(p, n_w, d) > 0.0]
    assert dirs, "the plane's normal selects at least one direction"
    J = math.ceil(2 * tau / vox - 1e-9)
    h = 2 * tau / J
    block = 8 * vox
    exact, long_enough = set(), set()
    # pixels with a valid cross-product normal: the image border has no four neighbours
    for v in range(1, H - 1):
        for u in range(1, W - 1):
            pc = (depth[v, u] / rays[v, u, 2]) * rays[v, u]
            pw = T[:3, :3] @ pc + T[:3, 3]
            rw = T[:3, :3] @ (pc / np.linalg.norm(pc))
            for key, length in segment_blocks(pw - tau * rw, pw + tau * rw, block).items():
                for d in dirs:
                    exact.add(key + (d,))
                    if length > h + 1e-9:
                        long_enough.add(key + (d,))
    # no other block than those the segments pass through ...
    assert requested - flagged <= exact, sorted(requested - flagged - exact)[:5]
    # ... and every block a segment crosses for more than the sample spacing
    missing = long_enough - requested - flagged
    assert not missing, sorted(missing)[:5]
    assert len(requested) > 50
