"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed forms (planes,
spheres), stated properties (direction weight), special cases (a single-direction map is a
regular TSDF; a plate seen from both sides), brute force (fine ray marching), textbook
identities (matrix exponential series, finite differences) and exact recovery problems.
"""
import math

import numpy as np
import pytest

import synth
from synth.scenes import Box, Camera, Scene, Sphere, render_frame, look_at
from oracle import oracle as O

TINY = synth.scenes.TINY_CAMERA


# ----------------------------------------------------------------------------------------
# Direction weight (Sec. 3, eq. direction_weight; properties stated right after it)
# ----------------------------------------------------------------------------------------

@pytest.mark.parametrize("theta", [math.pi / 3, 0.85, 1.2, math.pi / 2])
def test_direction_weight_properties(theta):
    P = O.MapParams(voxel=0.01, tau=0.04, theta=theta)
    theta = O.f32(theta)                 # parameters are float32 values on both sides
    lo, hi = math.pi / 2 - theta, theta
    alphas = np.linspace(0.0, math.pi, 721)
    for a in alphas:
        n = (math.cos(a), math.sin(a), 0.0)
        wx = O.w_dir(P, n, 0)
        wy = O.w_dir(P, n, 2)
        if a <= lo - 1e-12:
            assert wx == 1.0          # exclusive zone of X+
        if a >= hi + 1e-12:
            assert wx == 0.0          # beyond theta: no membership
        if a <= math.pi / 2:
            assert abs(wx + wy - 1.0) < 1e-12   # neighbouring axes share the blend zone
    # linear across the blend zone: vanishing second differences, end values 1 and 0
    zs = np.linspace(max(lo, 0.0), hi, 9)
    w = np.array([O.w_dir(P, (math.cos(a), math.sin(a), 0.0), 0) for a in zs])
    assert abs(w[-1]) < 1e-12
    if lo >= 0:
        assert abs(w[0] - 1) < 1e-12
    assert np.max(np.abs(w[:-2] - 2 * w[1:-1] + w[2:])) < 1e-12
    # half membership at 45 degrees
    n45 = (math.sqrt(0.5), math.sqrt(0.5), 0.0)
    assert abs(O.w_dir(P, n45, 0) - 0.5) < 1e-12


def test_every_normal_matches_one_to_three_directions():
    rng = np.random.default_rng(0)
    P = O.MapParams(voxel=0.01, tau=0.04)
    for _ in range(2000):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        k = sum(O.w_dir(P, n, d) > 0 for d in range(6))
        assert 1 <= k <= 3


# ----------------------------------------------------------------------------------------
# Planes: the point-to-plane SDF of a plane is exact (Sec. 3, eq. point-to-plane), and the
# trilinear interpolant reproduces a linear field, so rendering recovers the plane exactly.
# ----------------------------------------------------------------------------------------

def _voxel_positions(blob, voxel):
    keys = blob["keys"].astype(np.int64)
    l = np.arange(512)
    loc = np.stack([l % 8, (l // 8) % 8, l // 64], axis=1)
    idx = keys[:, None, :3] * 8 + loc[None]
    return idx * O.f32(voxel)


def _plane_depth(cam, T_wc, q, n):
    """Depth image of the plane through q with unit normal n (world), float32."""
    R, t = T_wc[:3, :3], T_wc[:3, 3]
    qc = R.T @ (q - t)
    nc = R.T @ n
    rays = cam.pixel_rays()
    z = (qc @ nc) / (rays @ nc)
    return np.where(z > 0, z, 0).astype(np.float32)


def test_frontal_plane_fusion_and_render_exact():
    cam = TINY
    T = np.eye(4)                                  # camera looks along world +z
    depth = np.full((cam.height, cam.width), 0.5, np.float32)
    rgb = np.zeros((cam.height, cam.width, 3), np.uint8)
    rgb[...] = (30, 140, 250)
    m = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04))
    m.integrate(depth, rgb, cam, T)
    b = m.export()
    assert set(b["keys"][:, 3].tolist()) == {5}    # only Z- holds a frontal plane facing -z
    x = _voxel_positions(b, 0.01)
    tau = O.f32(0.04)
    d_true = (0.5 - x[..., 2]) / tau
    w = b["w"]
    band = (w > 0) & (np.abs(d_true) <= 1)
    assert band.sum() > 10000
    assert np.max(np.abs(b["sdf"][band] - d_true[band])) < 1e-6      # float32 export
    # weight = w_angle = cosine between viewing ray and normal (w_dir = 1, w_depth = 1)
    cosang = x[..., 2] / np.linalg.norm(x, axis=-1)
    assert np.max(np.abs(w[band] - cosang[band])) < 5e-3
    # voxels in front of the band are carved to exactly 1 with the constant weight
    carved = (w > 0) & (d_true > 1)
    assert carved.sum() > 1000
    assert np.all(b["sdf"][carved] == 1.0) and np.all(np.abs(w[carved] - 0.1) < 1e-7)
    # voxels behind the band are never updated
    assert np.all(w[d_true < -1 - 1e-6] == 0)
    # uniform albedo is reproduced exactly; the colour weight vanishes beyond tau
    cw = b["wc"]
    assert np.all(b["rgb"][cw > 0] == np.array([30, 140, 250], np.uint8))
    assert np.all(cw[np.abs(d_true) > 1.0 + 1e-6] == 0)
    # render: interior pixels hit z = 0.5 with normal -z (camera frame), exactly; near the
    # image border the cells reach voxels that project outside the frame and stay empty
    o = m.render(cam, T)
    mask = o.mask.reshape(cam.height, cam.width)
    inner = np.zeros_like(mask, bool)
    inner[6:-6, 6:-6] = True
    assert np.all(mask[inner] == 1)
    dep = o.depth.reshape(cam.height, cam.width)
    assert np.max(np.abs(dep[inner] - 0.5)) < 1e-8
    nrm = o.normal.reshape(cam.height, cam.width, 3)[inner]
    assert np.max(np.abs(nrm - np.array([0, 0, -1.0]))) < 1e-9
    assert np.all(o.rgba.reshape(cam.height, cam.width, 4)[inner][:, :3] ==
                  np.array([30, 140, 250], np.uint8))


def test_oblique_plane_blend_zone():
    """Normal half-way between X- and Z-: both directions hold the same linear field with
    half the weight each (partition of unity); render recovers the plane."""
    cam = TINY
    T = np.eye(4)
    n = np.array([-1.0, 0.0, -1.0]) / math.sqrt(2.0)   # faces the camera
    q = np.array([0.0, 0.0, 0.6])
    depth = _plane_depth(cam, T, q, n)
    m = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04))
    m.integrate(depth, None, cam, T)
    b = m.export()
    dirs = set(b["keys"][:, 3].tolist())
    assert dirs == {1, 5}
    x = _voxel_positions(b, 0.01)
    tau = O.f32(0.04)
    d_true = ((x - q) @ n) / tau
    band = (b["w"] > 0) & (np.abs(d_true) <= 0.999)
    assert band.sum() > 5000
    assert np.max(np.abs(b["sdf"][band] - d_true[band])) < 2e-5
    # the two directions hold identical values and weights (w_dir = 1/2 each)
    kx = {tuple(k[:3]): i for i, k in enumerate(b["keys"]) if k[3] == 1}
    kz = {tuple(k[:3]): i for i, k in enumerate(b["keys"]) if k[3] == 5}
    common = sorted(set(kx) & set(kz))
    assert len(common) > 20
    ix = np.array([kx[c] for c in common])
    iz = np.array([kz[c] for c in common])
    # (normals from float32 depths deviate ~1e-5 rad from 45 degrees)
    assert np.max(np.abs(b["w"][ix] - b["w"][iz])) < 1e-4
    both = (b["w"][ix] > 0) & (b["w"][iz] > 0)
    assert np.max(np.abs(b["sdf"][ix][both] - b["sdf"][iz][both])) < 1e-6
    cosang = np.abs((x[ix] / np.linalg.norm(x[ix], axis=-1, keepdims=True)) @ n)
    sel = (b["w"][ix] > 0) & (np.abs(d_true[ix]) <= 1)
    assert np.max(np.abs(b["w"][ix][sel] - 0.5 * cosang[sel])) < 5e-3
    o = m.render(cam, T)
    rays = cam.pixel_rays().reshape(-1, 3)
    z_true = (q @ n) / (rays @ n)
    mask = o.mask.reshape(cam.height, cam.width)
    inner = np.zeros_like(mask, bool)
    inner[8:-8, 8:-8] = True
    inner = inner.ravel()
    hit = inner & (o.mask > 0)
    assert hit.sum() > 0.95 * inner.sum()
    assert np.max(np.abs(o.depth[hit] - z_true[hit])) < 2e-6
    assert np.max(np.abs(o.normal[hit] - n)) < 1e-4


# ----------------------------------------------------------------------------------------
# Sphere: closed-form depth within the discretisation error, second-order in the voxel size
# ----------------------------------------------------------------------------------------

def _sphere_error(voxel):
    """Median |rendered - analytic| depth on the cap of a sphere r = 0.2 m seen from +x.

    The ten fused views stay within 0.25 rad of the render direction: under oblique views
    the point-to-plane metric of Sec. 3 underestimates the distance to a curved surface by
    ~t^2 tan^2(beta) / (2 r) (t: distance along the view ray), so this pin keeps that term and
    the trilinear error both second order in the voxel size."""
    sc = Scene(spheres=[Sphere(np.zeros(3), 0.2, np.array([200, 80, 40], np.uint8))], boxes=[])
    cam = Camera(640, 480, 525.0, 525.0, 319.5, 239.5)
    rng = np.random.default_rng(1)
    m = O.OracleMap(O.MapParams(voxel=voxel, tau=0.04))
    for _ in range(10):
        a, b = rng.uniform(-0.25, 0.25, 2)
        eye = (math.cos(a) * math.cos(b), math.sin(a) * math.cos(b), math.sin(b))
        T = look_at(eye, (0, 0, 0))
        m.integrate(render_frame(sc, cam, T)["depth"], None, cam, T)
    c2 = Camera(160, 120, 120.0, 120.0, 79.5, 59.5)
    Tq = look_at((1.0, 0.05, 0.03), (0, 0, 0))
    f = render_frame(sc, c2, Tq)
    o = m.render(c2, Tq, z_far=2.0, classify=False)
    td = f["true_depth"].ravel()
    cap = (td > 0) & (np.abs(f["normal"].reshape(-1, 3)[:, 2]) > math.cos(math.radians(25)))
    hit = cap & (o.mask > 0)
    assert hit.sum() == cap.sum() > 400
    return np.median(np.abs(o.depth[hit] - td[hit]))


def test_sphere_depth_converges_second_order():
    e1, e2, e3 = _sphere_error(0.02), _sphere_error(0.01), _sphere_error(0.005)
    assert e2 < 1.5e-4 and e3 < 4e-5
    for r in (e1 / e2, e2 / e3):
        assert 3.0 < r < 5.5, (e1, e2, e3)


# ----------------------------------------------------------------------------------------
# Thin plate seen from both sides (Sec. 1 and Sec. 4: the DTSDF keeps both faces apart)
# ----------------------------------------------------------------------------------------

def _plate_map(single_direction=False):
    plate = Box(np.array([0.295, -0.30, -0.30]), np.array([0.305, 0.30, 0.30]),
                np.tile(np.array([90, 90, 90], np.uint8), (6, 1)))
    sc = Scene(spheres=[], boxes=[plate])
    m = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04, dense_lo=synth.scenes.TINY_DENSE_LO,
                                dense_hi=synth.scenes.TINY_DENSE_HI,
                                single_direction=single_direction))
    for phi in [-0.2, -0.1, 0.0, 0.1, 0.2]:
        for base in (0.0, math.pi):
            T = look_at((math.cos(base + phi), math.sin(base + phi), 0.0), (0, 0, 0))
            f = render_frame(sc, TINY, T)
            m.integrate(f["depth"], None, TINY, T)
    return m, sc


@pytest.mark.parametrize("base,face,nx", [(0.0, 0.305, 1.0), (math.pi, 0.295, -1.0)])
def test_thin_plate_renders_the_visible_face(base, face, nx):
    m, sc = _plate_map()
    T = look_at((math.cos(base + 0.05), math.sin(base + 0.05), 0.0), (0, 0, 0))
    o = m.render(TINY, T, z_far=2.5)
    f = render_frame(sc, TINY, T)
    inner = (f["true_depth"].ravel() > 0) & (np.abs(f["normal"].reshape(-1, 3)[:, 2]) > 0.9)
    # keep pixels whose hit is at least 3 cm inside the plate edges
    rays = TINY.pixel_rays().reshape(-1, 3)
    pw = (rays * f["true_depth"].reshape(-1, 1)) @ T[:3, :3].T + T[:3, 3]
    inner &= (np.abs(pw[:, 1]) < 0.27) & (np.abs(pw[:, 2]) < 0.27)
    assert inner.sum() > 500
    hit = inner & (o.mask > 0)
    assert hit.sum() == inner.sum()
    xw = (o.vertex[hit] @ T[:3, :3].T + T[:3, 3])[:, 0]
    assert np.max(np.abs(xw - face)) < 5e-4
    nw = o.normal[hit] @ T[:3, :3].T
    assert np.min(nw[:, 0] * nx) > math.cos(math.radians(3.0))


def test_thin_plate_fails_with_a_single_regular_tsdf():
    """Control: with one direction and no direction weighting the method is a regular TSDF,
    whose band cannot hold both faces of a plate thinner than the truncation distance."""
    m, sc = _plate_map(single_direction=True)
    T = look_at((math.cos(0.05), math.sin(0.05), 0.0), (0, 0, 0))
    o = m.render(TINY, T, z_far=2.5)
    f = render_frame(sc, TINY, T)
    inner = (f["true_depth"].ravel() > 0)
    hit = inner & (o.mask > 0)
    xw = (o.vertex[hit] @ T[:3, :3].T + T[:3, 3])[:, 0]
    assert np.median(np.abs(xw - 0.305)) > 5e-3


# ----------------------------------------------------------------------------------------
# Brute force: lattice probing + bracketed refinement equals the first crossing of a fine
# march of the same combined SDF (Sec. 4), on smooth random six-direction fields.
# ----------------------------------------------------------------------------------------

def _random_field_map(seed=5, voxel=0.01):
    rng = np.random.default_rng(seed)
    keys, sdf, w = [], [], []
    l = np.arange(512)
    loc = np.stack([l % 8, (l // 8) % 8, l // 64], axis=1).astype(np.float64)
    for bz in range(2):
        for by in range(2):
            for bx in range(2):
                for d in range(6):
                    keys.append((bx, by, bz, d))
    ph = rng.uniform(0, 2 * math.pi, (6, 4))
    fr = rng.uniform(0.15, 0.45, (6, 3))
    for (bx, by, bz, d) in keys:
        i = loc + 8 * np.array([bx, by, bz])
        v = (0.9 * np.sin(fr[d, 0] * i[:, 0] + ph[d, 0]) * np.cos(fr[d, 1] * i[:, 1] + ph[d, 1])
             + 0.4 * np.cos(fr[d, 2] * i[:, 2] + ph[d, 2]))
        sdf.append(np.clip(v, -1, 1))
        w.append(1.0 + 0.5 * np.sin(0.3 * i[:, 0] + 0.2 * i[:, 1] + ph[d, 3]))
    m = O.OracleMap(O.MapParams(voxel=voxel, tau=0.04, with_color=False))
    m.load(dict(keys=np.array(keys, np.int32), sdf=np.array(sdf, np.float32),
                w=np.array(w, np.float32)))
    return m


def test_lattice_march_matches_fine_march():
    m = _random_field_map()
    s = O.f32(0.01)
    step = O.f32(0.005)
    rng = np.random.default_rng(8)
    cam1 = Camera(1, 1, 100.0, 100.0, 0.0, 0.0)      # pixel (0,0) looks along camera +z
    agree = missed = 0
    for _ in range(24):
        c = np.array([0.08, 0.08, 0.08]) + rng.normal(size=3) * 0.02
        c += rng.normal(size=3) / np.linalg.norm(rng.normal(size=3)) * 0.0
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        eye = c - 0.3 * d
        T = look_at(eye, c, up=(0.3, 0.5, 0.8) if abs(d[2]) > 0.9 else (0, 0, 1))
        r = T[:3, 2]
        z_near, z_far = 0.05, 0.6
        o = m.render(cam1, T, pixels=np.array([[0, 0]]), z_near=z_near, z_far=z_far,
                     classify=False)
        # fine march of the same f at step 1e-4 voxel
        ts = np.arange(z_near, z_far, 1e-4 * s)
        f, dfn, _ = m.eval(eye + ts[:, None] * r, r)
        cross = np.nonzero(dfn[:-1] & dfn[1:] & (f[:-1] > 0) & (f[1:] <= 0))[0]
        if o.mask[0] == 0:
            # no lattice hit: every fine crossing must sit between lattice points of equal
            # sign (a pair of crossings inside one lattice interval)
            for j in cross:
                k = int(math.floor((ts[j] - z_near) / step))
                ta, tb = z_near + k * step, z_near + (k + 1) * step
                fab, dab, _ = m.eval(np.stack([eye + ta * r, eye + tb * r]), r)
                assert not (dab.all() and fab[0] > 0 and fab[1] <= 0)
            missed += len(cross) > 0
            continue
        assert len(cross) > 0
        a, b = ts[cross[0]], ts[cross[0] + 1]
        for _ in range(60):
            mid = 0.5 * (a + b)
            fm, dm, _ = m.eval((eye + mid * r)[None], r)
            if (not dm[0]) or fm[0] > 0:
                a = mid
            else:
                b = mid
        t_fine = 0.5 * (a + b)
        if abs(t_fine - o.thit[0]) < 1e-7:
            agree += 1
        else:
            # the fine march found an earlier crossing inside a lattice interval whose ends
            # do not bracket it
            assert t_fine < o.thit[0]
            k = int(math.floor((t_fine - z_near) / step))
            ta, tb = z_near + k * step, z_near + (k + 1) * step
            fab, dab, _ = m.eval(np.stack([eye + ta * r, eye + tb * r]), r)
            assert not (dab.all() and fab[0] > 0 and fab[1] <= 0)
            missed += 1
    assert agree >= 12, (agree, missed)


def test_trilinear_value_and_gradient_reproduce_trilinear_fields():
    """Phi^D of a single direction is the trilinear interpolant: a field that is itself
    trilinear in the voxel coordinates is reproduced exactly, and the hit of the combined
    SDF of one direction lies on its zero set."""
    keys = [(0, 0, 0, 5), (1, 0, 0, 5), (0, 1, 0, 5), (1, 1, 0, 5), (0, 0, 1, 5), (1, 0, 1, 5),
            (0, 1, 1, 5), (1, 1, 1, 5)]
    l = np.arange(512)
    loc = np.stack([l % 8, (l // 8) % 8, l // 64], axis=1).astype(np.float64)
    sdf = []
    for (bx, by, bz, _) in keys:
        i = loc + 8 * np.array([bx, by, bz])
        # decreasing along +z with a bilinear xy term: Z- faces the camera at -z
        sdf.append(np.clip(0.9 - 0.1 * i[:, 2] + 0.002 * i[:, 0] * i[:, 1], -1, 1))
    m = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04, with_color=False))
    m.load(dict(keys=np.array(keys, np.int32), sdf=np.array(sdf, np.float32),
                w=np.ones((8, 512), np.float32)))
    rng = np.random.default_rng(1)
    s = O.f32(0.01)
    pts = rng.uniform(0.02, 0.13, (200, 3))
    f, d, _ = m.eval(pts, np.array([0, 0, 1.0]))
    vi = pts / s
    exact = np.clip(0.9 - 0.1 * vi[:, 2] + 0.002 * vi[:, 0] * vi[:, 1], -1, 1)
    inside = (0.9 - 0.1 * vi[:, 2] + 0.002 * vi[:, 0] * vi[:, 1] < 0.95) & \
             (0.9 - 0.1 * vi[:, 2] + 0.002 * vi[:, 0] * vi[:, 1] > -0.95)
    assert d.all()
    # float32 storage of the voxel values bounds the agreement
    assert np.max(np.abs(f[inside] - exact[inside])) < 1e-6


# ----------------------------------------------------------------------------------------
# Fusion invariants (Sec. 3: weighted cumulative moving average; carving guard)
# ----------------------------------------------------------------------------------------

def test_fusing_twice_doubles_weights_and_keeps_values():
    cam = TINY
    T = np.eye(4)
    depth = np.full((cam.height, cam.width), 0.5, np.float32)
    m1 = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04))
    m2 = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04))
    m1.integrate(depth, None, cam, T)
    m2.integrate(depth, None, cam, T)
    m2.integrate(depth, None, cam, T)
    a, b = m1.export(), m2.export()
    assert np.array_equal(a["keys"], b["keys"])
    np.testing.assert_allclose(b["sdf"], a["sdf"], atol=1e-7)
    np.testing.assert_allclose(b["w"], np.minimum(2 * a["w"], 63.75), rtol=1e-6)
    for _ in range(700):          # the cap holds
        m1.integrate(depth, None, cam, T)
    assert m1.export()["w"].max() <= 63.75


def test_carving_is_suppressed_next_to_depth_jumps():
    """A voxel in free space is carved only if no depth within two pixels differs from the
    associated depth by more than tau (Sec. 3)."""
    cam = TINY
    T = np.eye(4)
    depth = np.full((cam.height, cam.width), 0.8, np.float32)
    depth[:, 80:] = 0.5            # step edge between columns 79 and 80
    m = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04))
    m.integrate(depth, None, cam, T)
    b = m.export()
    x = _voxel_positions(b, 0.01)
    u = cam.fx * x[..., 0] / x[..., 2] + cam.cx
    v = cam.fy * x[..., 1] / x[..., 2] + cam.cy
    ui, vi = np.floor(u + 0.5), np.floor(v + 0.5)
    inb = (ui >= 3) & (ui < cam.width - 3) & (vi >= 3) & (vi < cam.height - 3) & (x[..., 2] > 0)
    zpix = np.where(ui >= 80, 0.5, 0.8)
    free = inb & ((zpix - x[..., 2]) / O.f32(0.04) > 1.0 + 1e-6)
    near_edge = np.abs(ui - 79.5) <= 1.5      # the other side lies within two pixels
    far_edge = np.abs(ui - 79.5) >= 2.5
    carved = (b["sdf"] == 1.0) & (b["w"] == np.float32(0.1))   # the carving signature
    assert (free & near_edge).sum() > 100
    assert not np.any(carved[free & near_edge])              # never carved next to the jump
    carved_far = free & far_edge
    assert carved_far.sum() > 100 and np.all(carved[carved_far])


# ----------------------------------------------------------------------------------------
# Registration (Sec. 5, Sec. 6)
# ----------------------------------------------------------------------------------------

def _series_expm(G, terms=60):
    out = np.eye(4)
    term = np.eye(4)
    for k in range(1, terms):
        term = term @ G / k
        out = out + term
    return out


def test_exp_maps_textbook():
    rng = np.random.default_rng(2)
    for _ in range(20):
        xi = rng.normal(size=7) * np.array([0.3, 0.3, 0.3, 0.7, 0.7, 0.7, 0.2])
        E6 = O.exp_map(xi[:6])
        E7 = O.exp_map(xi)
        np.testing.assert_allclose(E6, _series_expm(O.generator(xi[:6])), atol=1e-13)
        np.testing.assert_allclose(E7, _series_expm(O.generator(xi)), atol=1e-13)
        # rotation part: Rodrigues' formula
        w = xi[3:6]
        th = np.linalg.norm(w)
        K = O.hat(w / th)
        Rr = np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K
        np.testing.assert_allclose(E6[:3, :3], Rr, atol=1e-13)
        np.testing.assert_allclose(E7[:3, :3], math.exp(xi[6]) * Rr, atol=1e-13)
        # one-parameter subgroup
        np.testing.assert_allclose(O.exp_map(0.3 * xi) @ O.exp_map(0.7 * xi), E7, atol=1e-12)
    # pure translation
    np.testing.assert_allclose(O.exp_map(np.array([1.0, 2, 3, 0, 0, 0]))[:3, 3], [1, 2, 3])


def test_point_to_plane_jacobian_matches_finite_differences():
    """J_i of eq. ICP_geometric_dx and the Sim(3) column of eq. sim3_derivative against
    central differences of r(xi) = <q - exp(xi) dT p, n>."""
    rng = np.random.default_rng(3)
    dT = O.exp_map(rng.normal(size=7) * 0.1)
    for dim in (6, 7):
        for _ in range(10):
            p = rng.normal(size=3)
            q = rng.normal(size=3)
            n = rng.normal(size=3)
            n /= np.linalg.norm(n)

            def r(xi):
                E = O.exp_map(xi) @ dT
                return (q - (E[:3, :3] @ p + E[:3, 3])) @ n

            y = dT[:3, :3] @ p + dT[:3, 3]
            J = np.concatenate([-n, -np.cross(y, n)] + ([[-(n @ y)]] if dim == 7 else []))
            h = 1e-6
            fd = np.array([(r(h * e) - r(-h * e)) / (2 * h) for e in np.eye(dim)])
            np.testing.assert_allclose(J, fd, atol=1e-8)


def _box_world():
    rng = np.random.default_rng(21)
    boxes = [Box(np.array([0.5, 0.4, 0.0]), np.array([1.1, 0.9, 0.7]),
                 np.tile(np.array([100, 100, 100], np.uint8), (6, 1))),
             Box(np.array([2.6, 2.9, 0.0]), np.array([3.3, 3.5, 1.2]),
                 np.tile(np.array([100, 100, 100], np.uint8), (6, 1))),
             Box(np.array([0.6, 2.8, 0.9]), np.array([1.2, 3.4, 1.3]),
                 np.tile(np.array([100, 100, 100], np.uint8), (6, 1)))]
    del rng
    return Scene(spheres=[], boxes=boxes,
                 room=synth.scenes.Room(np.zeros(3), np.array([4.0, 4.0, 3.0]),
                                        np.tile(np.array([50, 50, 50], np.uint8), (6, 1))))


def _model_levels(sc, cam, T, L=3):
    out = []
    for l in range(L):
        c = cam.level(l)
        f = render_frame(sc, c, T)
        V = c.pixel_rays() * f["true_depth"][..., None]
        out.append((V, f["normal"], f["hit"].astype(np.uint8), c))
    return out


def test_icp_recovers_exact_offset_on_planar_scene():
    """Noise-free planar scene: point-to-plane ICP with projective association converges to
    the true relative pose (P7)."""
    sc = _box_world()
    cam = Camera(640, 480, 525.0, 525.0, 319.5, 239.5)
    T = synth.room_pose(40)
    live = render_frame(sc, cam, T)["depth"]
    rng = np.random.default_rng(4)
    dT0 = synth.perturb_pose(0.02, math.radians(2.0), rng)
    dT, log = O.icp(live, cam, _model_levels(sc, cam, T), dT0, dim=6, iters=(20, 10, 10))
    assert np.max(np.abs(dT - np.eye(4))) < 1e-6, log[-1]


@pytest.mark.parametrize("s", [0.93, 1.0, 1.07])
def test_sim3_icp_recovers_depth_scale(s):
    """A sensor whose depth is scaled by s registers with exp(sigma) = 1/s (Sec. 6,
    eq. reprojection: scaling the depth is scaling the point)."""
    sc = _box_world()
    cam = Camera(640, 480, 525.0, 525.0, 319.5, 239.5)
    T = synth.room_pose(40)
    live = render_frame(sc, cam, T, depth_scale=s)["depth"]
    rng = np.random.default_rng(6)
    dT0 = synth.perturb_pose(0.01, math.radians(1.0), rng)
    # the prior carries a scale estimate within 1.5% (Sec. 6 starts from a visually close
    # scale); a 10% scale error would push most points past the 10 cm rejection distance
    dT0[:3, :3] *= 1.015 / s
    dT, log = O.icp(live, cam, _model_levels(sc, cam, T), dT0, dim=7, iters=(30, 15, 15))
    sR = dT[:3, :3]
    scale = np.cbrt(np.linalg.det(sR))
    assert abs(scale - 1.0 / s) < 1e-6, (scale, 1 / s)
    np.testing.assert_allclose(sR / scale, np.eye(3), atol=1e-6)
    np.testing.assert_allclose(dT[:3, 3], 0, atol=1e-6)


def test_normal_equations_solution_is_stationary():
    """The Cholesky step zeroes the gradient of the linearised error (eq. ICP_solution)."""
    rng = np.random.default_rng(9)
    J = rng.normal(size=(1000, 7))
    r = rng.normal(size=1000)
    H = J.T @ J
    g = J.T @ r
    xi = O.solve_step(H, g)
    assert np.max(np.abs(J.T @ (J @ xi + r))) < 1e-9


# ----------------------------------------------------------------------------------------
# Precision form: stored codes are the nearest float16 / int16 / uint8 values
# ----------------------------------------------------------------------------------------

@pytest.mark.parametrize("sdf_fmt", [1, 2])
def test_quantised_storage_matches_reference_rounding(sdf_fmt):
    """A single frontal-plane frame: each stored distance is the round-half-even code of the
    exact distance (numpy's float16 conversion / numpy.rint), weights are multiples of 1/4."""
    cam = TINY
    T = np.eye(4)
    depth = np.full((cam.height, cam.width), 0.5, np.float32)
    m = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04, sdf_fmt=sdf_fmt, w_fmt=1, w_carve=0.5))
    m.integrate(depth, None, cam, T)
    b = m.export()
    x = _voxel_positions(b, 0.01)
    tau = O.f32(0.04)
    d_true = (0.5 - x[..., 2]) / tau
    band = (b["w"] > 0) & (np.abs(d_true) <= 1)
    assert band.sum() > 10000
    if sdf_fmt == 1:
        expect = d_true[band].astype(np.float16).astype(np.float64)
    else:
        # the code times the float32 scale 1/32767, product rounded to float32
        expect = (np.rint(d_true[band] * 32767.0).astype(np.float32) *
                  np.float32(1.0 / 32767.0)).astype(np.float64)
        assert np.mean(b["sdf"][band] == expect) > 0.999
    assert np.max(np.abs(b["sdf"][band] - expect)) < 1e-7      # float32 export of the code
    q = np.sqrt(b["w"] * 1024.0)
    assert np.all(q == np.round(q)) and q.max() <= 255
    # weights are the coded view cosines of the pixel rays (one frame); the voxel's own
    # viewing direction differs from its pixel's ray by up to half a pixel, so within one
    # code step of the code of its cosine
    cosang = x[..., 2] / np.linalg.norm(x, axis=-1)
    qe = np.minimum(np.rint(np.sqrt(1024.0 * cosang[band])), 255)
    assert np.all(np.abs(b["w"][band] - qe ** 2 / 1024.0) <= (2 * qe + 1) / 1024.0)


def _weight_code(w):
    """The uint8 weight code written out: q = round-half-even(sqrt(1024 w)), at most 255."""
    return int(min(255, np.rint(math.sqrt(1024.0 * w))))


def test_weight_code_definition():
    """Values the square-law code fixes: 0 and the top, the exact code points, a tie
    between two codes going to the even one, and the step at small weights."""
    m = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04, w_fmt=1))
    del m
    assert _weight_code(0.0) == 0 and _weight_code(63.5) == 255 and _weight_code(100.0) == 255
    for q in (1, 7, 100, 254):
        assert _weight_code(q * q / 1024.0) == q
    # (q + 1/2)^2 / 1024 lies halfway between codes q and q + 1 in the square root
    assert _weight_code((10.5 ** 2) / 1024.0) == 10 and _weight_code((11.5 ** 2) / 1024.0) == 12
    # a carving weight of 0.1 is representable to within 1 %
    assert abs(_weight_code(0.1) ** 2 / 1024.0 - 0.1) < 0.003


@pytest.mark.parametrize("sdf_fmt", [1, 2])
def test_quantised_weights_accumulate(sdf_fmt):
    """Repeated carving (w_carve = 0.1) and repeated small fusion weights raise the stored
    uint8 weight frame after frame, as the float32 weights do, instead of rounding back
    to the old code: the cumulative weighted average of Sec. 3 is kept."""
    cam = TINY
    T = np.eye(4)
    # a frontal plane at 0.5 m seen through a thin slab of voxels: voxels in front of the
    # band are carved, voxels in the band are fused with the view cosine as weight
    depth = np.full((cam.height, cam.width), 0.5, np.float32)
    plain = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04))
    packed = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04, sdf_fmt=sdf_fmt, w_fmt=1))
    wp, wq = [], []
    for _ in range(6):
        plain.integrate(depth, None, cam, T)
        packed.integrate(depth, None, cam, T)
        bp, bq = plain.export(), packed.export()
        assert np.array_equal(bp["keys"], bq["keys"])
        wp.append(bp["w"].copy())
        wq.append(bq["w"].copy())
    x = _voxel_positions(bp, 0.01)
    d = (0.5 - x[..., 2]) / O.f32(0.04)
    carved = (d > 1.2) & (wp[-1] > 0)
    band = (np.abs(d) < 0.8) & (wp[-1] > 0)
    assert carved.sum() > 1000 and band.sum() > 1000
    for sel in (carved, band):
        for k in range(1, 6):
            # every frame raises every stored weight ...
            assert np.all(wq[k][sel] > wq[k - 1][sel])
            # ... and each of the k + 1 updates so far rounded by at most half a code step
            step = (2.0 * np.sqrt(wq[k][sel] * 1024.0) + 1.0) / 1024.0
            assert np.all(np.abs(wq[k][sel] - wp[k][sel]) <= (k + 1) * step / 2)
