"""Pins of the oracle's view-dependent combined ("rendering") TSDF and of conditional
recombination (Sec. 4: Lemma positional_unambiguity, the precomputed combined TSDF,
eq. condition_1 .. condition_4; Sec. 7: integer-position evaluation with six-neighbour
gradients).

The combined TSDF is checked against closed forms (planes, linear fields whose central
differences are exact, the 45-degree partition of unity), the special structure of a thin
plate (each side's volume holds the face visible from that side), brute-force projection of
every voxel for the frustum, and the definition of the rotation angle for the policy.
"""
import math

import numpy as np
import pytest

import synth
from synth.scenes import Camera, look_at, random_rotation_small, render_frame
from oracle import oracle as O

from tests.test_oracle_pins import _plate_map, _plane_depth, _voxel_positions

TINY = synth.scenes.TINY_CAMERA


def _combined(src_params: O.MapParams) -> O.OracleMap:
    p = O.MapParams(voxel=src_params.voxel, tau=src_params.tau, theta=src_params.theta,
                    step=src_params.step, with_color=src_params.with_color,
                    single_direction=True)
    return O.OracleMap(p)


def _index(blob):
    return {tuple(k[:3]): i for i, k in enumerate(blob["keys"])}


# ----------------------------------------------------------------------------------------
# Planes: every direction holding the plane holds the same linear field, so the combined
# value is that field and the combined TSDF renders the plane exactly.
# ----------------------------------------------------------------------------------------

def test_frontal_plane_combined_tsdf_is_exact():
    cam = TINY
    T = np.eye(4)
    depth = np.full((cam.height, cam.width), 0.5, np.float32)
    rgb = np.zeros((cam.height, cam.width, 3), np.uint8)
    rgb[...] = (30, 140, 250)
    src = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04))
    src.integrate(depth, rgb, cam, T)
    dst = _combined(src.params)
    dst.combine(src, cam, T)
    b = dst.export()
    assert set(b["keys"][:, 3].tolist()) == {0}
    assert len(b["keys"]) == len({tuple(k[:3]) for k in src.export()["keys"]})
    x = _voxel_positions(b, 0.01)
    tau = O.f32(0.04)
    d_true = (0.5 - x[..., 2]) / tau
    sb = src.export()
    si = _index(sb)
    w_src = np.zeros_like(b["w"])
    for k, i in _index(b).items():
        w_src[i] = sb["w"][si[k]]
    # observed voxels inside the band: the combined value is the signed distance
    band = (b["w"] > 0) & (np.abs(d_true) <= 0.999)
    assert band.sum() > 8000
    assert np.max(np.abs(b["sdf"][band] - d_true[band])) < 1e-6
    # carved voxels (value 1, zero gradient): fallback weights, value 1
    carved = (b["w"] > 0) & (d_true > 1.3)
    assert carved.sum() > 1000 and np.all(b["sdf"][carved] == 1.0)
    # unobserved voxels hold no value; observed ones always get one here
    assert np.all(b["w"][w_src == 0] == 0)
    assert np.all(b["w"][(w_src > 0) & (b["border"] == 0)] == 1)
    # uniform albedo
    assert np.all(b["rgb"][b["wc"] > 0] == np.array([30, 140, 250], np.uint8))
    o = dst.render(cam, T)
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


def test_oblique_plane_combined_tsdf():
    """Normal half-way between X- and Z-: both directions hold the plane's field, so the
    combined field is the plane's and the combined TSDF renders the plane."""
    cam = TINY
    T = np.eye(4)
    n = np.array([-1.0, 0.0, -1.0]) / math.sqrt(2.0)
    q = np.array([0.0, 0.0, 0.6])
    src = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04))
    src.integrate(_plane_depth(cam, T, q, n), None, cam, T)
    dst = _combined(src.params)
    dst.combine(src, cam, T)
    b = dst.export()
    x = _voxel_positions(b, 0.01)
    d_true = ((x - q) @ n) / O.f32(0.04)
    band = (b["w"] > 0) & (np.abs(d_true) <= 0.95)
    assert band.sum() > 4000
    assert np.max(np.abs(b["sdf"][band] - d_true[band])) < 2e-5
    o = dst.render(cam, T)
    rays = cam.pixel_rays().reshape(-1, 3)
    z_true = (q @ n) / (rays @ n)
    inner = np.zeros((cam.height, cam.width), bool)
    inner[8:-8, 8:-8] = True
    inner = inner.ravel()
    hit = inner & (o.mask > 0)
    assert hit.sum() > 0.95 * inner.sum()
    assert np.max(np.abs(o.depth[hit] - z_true[hit])) < 2e-6
    assert np.max(np.abs(o.normal[hit] - n)) < 1e-4


# ----------------------------------------------------------------------------------------
# Linear fields: central differences of a linear field are exact, so every weight factor of
# eq. combine_weight is known in closed form.
# ----------------------------------------------------------------------------------------

def _linear_field_map(g, offsets, weights, observed=None, voxel=0.01):
    """2x2x2 blocks; direction d holds Phi_d(x) = <x, g_d> + offsets[d] (x in voxels) with
    weight weights[d] (directions with weight 0 are absent); ``observed(d, idx)`` may clear
    voxels."""
    keys, sdf, w = [], [], []
    l = np.arange(512)
    loc = np.stack([l % 8, (l // 8) % 8, l // 64], axis=1).astype(np.float64)
    for bz in range(2):
        for by in range(2):
            for bx in range(2):
                idx = loc + 8 * np.array([bx, by, bz])
                for d in range(6):
                    if weights[d] == 0:
                        continue
                    keys.append((bx, by, bz, d))
                    sdf.append(idx @ g[d] + offsets[d])
                    ww = np.full(512, float(weights[d]))
                    if observed is not None:
                        ww = np.where(observed(d, idx), ww, 0.0)
                    w.append(ww)
    m = O.OracleMap(O.MapParams(voxel=voxel, tau=0.04, with_color=False))
    m.load(dict(keys=np.array(keys, np.int32), sdf=np.array(sdf, np.float32),
                w=np.array(w, np.float32)))
    return m


def _value_at(blob, v):
    b = tuple(int(c) // 8 for c in v)
    i = _index(blob)[b]
    l = (v[0] % 8) + 8 * (v[1] % 8) + 64 * (v[2] % 8)
    return blob["sdf"][i, l], blob["w"][i, l]


def test_combined_value_of_linear_fields_closed_form():
    s = 0.01
    gh = np.array([-1.0, 0.0, -1.0]) / math.sqrt(2.0)   # 45 deg between X- and Z-
    g = [None] * 6
    g[1] = g[5] = 0.03 * gh                 # X-, Z-: the visible surface, w_dir = 1/2 each
    g[0] = -0.03 * gh                       # X+: faces away from the camera
    g[2] = g[3] = g[4] = 0.03 * gh          # Y+, Y-, Z+: w_dir(gh) = 0
    offsets = [0.5, -0.25, 0.125, -0.375, 0.0625, 0.2]
    weights = [3.0, 1.0, 2.0, 2.0, 5.0, 4.0]
    src = _linear_field_map(g, offsets, weights)
    # camera on the side the normal gh points to, looking back at the voxels
    centre = np.array([8.0, 8.0, 8.0]) * s + 0.6 * gh
    T = look_at(centre, np.array([8.0, 8.0, 8.0]) * s, up=(0.0, 1.0, 0.0))
    dst = _combined(src.params)
    dst.combine(src, Camera(64, 64, 30.0, 30.0, 31.5, 31.5), T)
    b = dst.export()
    for v in [(5, 6, 7), (8, 8, 8), (10, 9, 6), (6, 10, 10)]:
        x = np.array(v, np.float64)
        phi = {d: x @ g[d] + offsets[d] for d in range(6)}
        # w_dir(gh) = 1/2 for X- and Z- (45 degrees, pinned by the direction-weight test),
        # their view cosines are equal, so the combination is the W-weighted mean
        expect = (weights[1] * phi[1] + weights[5] * phi[5]) / (weights[1] + weights[5])
        f, w = _value_at(b, v)
        assert w == 1
        assert abs(f - np.float32(expect)) < 1e-6, (v, f, expect)


def test_direction_without_six_observed_neighbours_leaves_the_gradient_branch():
    s = 0.01
    gh = np.array([-1.0, 0.0, -1.0]) / math.sqrt(2.0)
    g = [None, 0.03 * gh, None, None, None, 0.03 * gh]
    offsets = [0, -0.25, 0, 0, 0, 0.2]
    weights = [0, 1.0, 0, 0, 0, 4.0]
    # X- unobserved on the slab x index == 9
    src = _linear_field_map(g, offsets, weights, observed=lambda d, i: ~((d == 1) & (i[:, 0] == 9)))
    centre = np.array([8.0, 8.0, 8.0]) * s + 0.6 * gh
    T = look_at(centre, np.array([8.0, 8.0, 8.0]) * s, up=(0.0, 1.0, 0.0))
    dst = _combined(src.params)
    dst.combine(src, Camera(64, 64, 30.0, 30.0, 31.5, 31.5), T)
    b = dst.export()
    for v in [(8, 7, 7), (10, 6, 9)]:       # a neighbour of these lies on the slab
        x = np.array(v, np.float64)
        f, w = _value_at(b, v)
        assert w == 1 and abs(f - np.float32(x @ g[5] + offsets[5])) < 1e-6
    x = np.array((6, 7, 7), np.float64)      # away from the slab: both directions
    f, _ = _value_at(b, (6, 7, 7))
    expect = ((x @ g[1] + offsets[1]) * 1.0 + (x @ g[5] + offsets[5]) * 4.0) / 5.0
    assert abs(f - np.float32(expect)) < 1e-6


def test_backfacing_only_voxels_use_the_fallback_weights():
    """Only X+ is present and its gradient faces away from the camera: the gradient weights
    vanish, and eq. combine_tsdf_weight with <v^X+, -r> > 0 returns the X+ value."""
    s = 0.01
    g = [np.array([-0.03, 0.0, 0.0]), None, None, None, None, None]
    src = _linear_field_map(g, [0.3, 0, 0, 0, 0, 0], [2.0, 0, 0, 0, 0, 0])
    centre = np.array([8.0, 8.0, 8.0]) * s + np.array([0.6, 0.0, 0.0])
    T = look_at(centre, np.array([8.0, 8.0, 8.0]) * s)
    dst = _combined(src.params)
    dst.combine(src, Camera(64, 64, 30.0, 30.0, 31.5, 31.5), T)
    b = dst.export()
    for v in [(7, 8, 8), (9, 6, 10)]:
        f, w = _value_at(b, v)
        assert w == 1 and abs(f - np.float32(np.array(v, float) @ g[0] + 0.3)) < 1e-6
    # seen from the other side, <v^X+, -r> < 0 as well: no value
    T2 = look_at(np.array([8.0, 8.0, 8.0]) * s - np.array([0.6, 0.0, 0.0]),
                 np.array([8.0, 8.0, 8.0]) * s)
    dst2 = _combined(src.params)
    dst2.combine(src, Camera(64, 64, 30.0, 30.0, 31.5, 31.5), T2)
    _, w = _value_at(dst2.export(), (7, 8, 8))
    assert w == 0


# ----------------------------------------------------------------------------------------
# Thin plate (Lemma positional_unambiguity): from each side the combined TSDF holds the face
# visible from there, and a volume combined for one side is wrong for the other.
# ----------------------------------------------------------------------------------------

def _plate_inner(sc, T):
    f = render_frame(sc, TINY, T)
    inner = (f["true_depth"].ravel() > 0) & (np.abs(f["normal"].reshape(-1, 3)[:, 2]) > 0.9)
    rays = TINY.pixel_rays().reshape(-1, 3)
    pw = (rays * f["true_depth"].reshape(-1, 1)) @ T[:3, :3].T + T[:3, 3]
    return inner & (np.abs(pw[:, 1]) < 0.27) & (np.abs(pw[:, 2]) < 0.27)


@pytest.mark.parametrize("base,face,nx", [(0.0, 0.305, 1.0), (math.pi, 0.295, -1.0)])
def test_thin_plate_combined_tsdf_holds_the_visible_face(base, face, nx):
    src, sc = _plate_map()
    T = look_at((math.cos(base + 0.05), math.sin(base + 0.05), 0.0), (0, 0, 0))
    dst = _combined(src.params)
    dst.combine(src, TINY, T)
    o = dst.render(TINY, T, z_far=2.5)
    inner = _plate_inner(sc, T)
    assert inner.sum() > 500
    hit = inner & (o.mask > 0)
    assert hit.sum() == inner.sum()
    xw = (o.vertex[hit] @ T[:3, :3].T + T[:3, 3])[:, 0]
    assert np.max(np.abs(xw - face)) < 5e-4
    nw = o.normal[hit] @ T[:3, :3].T
    assert np.min(nw[:, 0] * nx) > math.cos(math.radians(3.0))


def test_thin_plate_combined_value_depends_on_the_viewpoint():
    src, sc = _plate_map()
    TA = look_at((1.0, 0.0, 0.0), (0, 0, 0))
    TB = look_at((-1.0, 0.0, 0.0), (0, 0, 0))
    A, B = _combined(src.params), _combined(src.params)
    A.combine(src, TINY, TA)
    B.combine(src, TINY, TB)
    ba, bb = A.export(), B.export()
    # voxel x = 0.29 (0.5 cm outside the -x face, 1.5 cm behind the +x face)
    for y in (-5, 0, 7):
        for z in (-6, 2):
            fa, wa = _value_at(ba, (29, y, z))
            fb, wb = _value_at(bb, (29, y, z))
            assert wa == 1 and wb == 1
            assert abs(fa - (-0.375)) < 2e-3          # occupied, seen from +x
            assert abs(fb - 0.125) < 2e-3             # free space, seen from -x
    # the +x volume rendered from -x does not show the -x face
    o = A.render(TINY, TB, z_far=2.5)
    inner = _plate_inner(sc, TB)
    hit = inner & (o.mask > 0)
    xw = (o.vertex[hit] @ TB[:3, :3].T + TB[:3, 3])[:, 0] if hit.any() else np.zeros(1) + 1.0
    assert hit.sum() < 0.5 * inner.sum() or np.median(np.abs(xw - 0.295)) > 5e-3


# ----------------------------------------------------------------------------------------
# Frustum selection (the image widened by 1/8 of its size per side, Sec. 4) by brute force
# ----------------------------------------------------------------------------------------

def _random_map(seed=5):
    rng = np.random.default_rng(seed)
    keys, sdf, w = [], [], []
    for bz in range(-2, 2):
        for by in range(-2, 2):
            for bx in range(-2, 2):
                for d in range(6):
                    keys.append((bx, by, bz, d))
                    sdf.append(rng.uniform(-1, 1, 512))
                    w.append(rng.uniform(0.5, 2.0, 512))
    m = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04, with_color=False))
    m.load(dict(keys=np.array(keys, np.int32), sdf=np.array(sdf, np.float32),
                w=np.array(w, np.float32)))
    return m


def _projects_inside(x, T, cam, margin):
    y = (x - T[:3, 3]) @ T[:3, :3]
    z = y[..., 2]
    zz = np.where(z > 0, z, 1.0)
    u = cam.fx * y[..., 0] / zz + cam.cx
    v = cam.fy * y[..., 1] / zz + cam.cy
    W, H = cam.width, cam.height
    return (z > 0) & (u >= -0.5 - margin * W) & (u < W - 0.5 + margin * W) & \
        (v >= -0.5 - margin * H) & (v < H - 0.5 + margin * H)


@pytest.mark.parametrize("margin", [0.0, 0.125])
def test_frustum_selection_brute_force(margin):
    src = _random_map()
    cam = Camera(40, 30, 80.0, 80.0, 19.5, 14.5)
    T = look_at((0.35, -0.12, 0.2), (0.02, 0.01, -0.03))
    dst = _combined(src.params)
    dst.combine(src, cam, T, margin=margin)
    b = dst.export()
    x = _voxel_positions(b, 0.01)
    inside = _projects_inside(x, T, cam, margin)
    sure = (b["border"] & 1) == 0
    assert 0.05 < inside.mean() < 0.95
    # every voxel is observed in all six directions, so every voxel in the frustum has a
    # value (some direction always has <v^D, -r> > 0) and no other voxel has one
    assert np.array_equal(b["w"][sure] > 0, inside[sure])


def test_fill_evaluates_only_voxels_without_value():
    src = _random_map()
    cam = Camera(40, 30, 80.0, 80.0, 19.5, 14.5)
    T1 = look_at((0.35, -0.12, 0.2), (0.02, 0.01, -0.03))
    T2 = look_at((0.30, 0.05, 0.25), (-0.05, 0.0, 0.0))
    dst = _combined(src.params)
    dst.combine(src, cam, T1)
    before = dst.export()
    dst.combine(src, cam, T1, T_frustum=T2, margin=0.0, only_missing=True)
    after = dst.export()
    had = before["w"] > 0
    assert np.array_equal(after["sdf"][had], before["sdf"][had])
    x = _voxel_positions(after, 0.01)
    in2 = _projects_inside(x, T2, cam, 0.0)
    sure = (after["border"] & 1) == 0
    new = ~had & in2 & sure
    assert new.sum() > 100
    # the new values are the combined values for the camera centre of T1
    ref = _combined(src.params)
    ref.combine(src, cam, T1, T_frustum=T2, margin=0.0)
    rb = ref.export()
    assert np.array_equal(after["sdf"][new], rb["sdf"][new])
    assert np.all(after["w"][new] == 1)
    assert np.all(after["w"][~had & ~in2 & sure] == 0)


# ----------------------------------------------------------------------------------------
# Conditional recombination (eq. condition_1 .. condition_4)
# ----------------------------------------------------------------------------------------

def test_rotation_angle_definition():
    rng = np.random.default_rng(2)
    for a in [1e-4, 0.01, 0.0785, 0.5, 2.0, 3.0]:
        ax = rng.normal(size=3)
        R = random_rotation_small(ax, a)
        assert abs(O.rotation_angle(R) - a) < 1e-9


def _pose(t=(0, 0, 0), axis=(0, 0, 1), angle=0.0):
    T = np.eye(4)
    T[:3, :3] = random_rotation_small(np.array(axis, float), angle)
    T[:3, 3] = t
    return T


def test_recombination_conditions():
    P = O.RecombinePolicy()
    base = _pose((1.0, 2.0, 0.5), (0.3, 1.0, -0.2), 0.7)
    # boot up: the first five frames always recombine
    assert [P.decide(base) for _ in range(5)] == [True] * 5
    # a static camera recombines again once more than 50 frames have passed
    seq = [P.decide(base) for _ in range(60)]
    assert seq.index(True) == 50           # frames since the last update: 51 > 50
    assert not any(seq[51:])
    # translation: 0.05 m is not enough, 0.0501 m is
    Q = O.RecombinePolicy(boot_frames=1)
    assert Q.decide(base)
    step = np.array([0.6, -0.8, 0.0])
    Tt = base.copy()
    Tt[:3, 3] += 0.0499 * step
    assert not Q.decide(Tt)
    Tt[:3, 3] = base[:3, 3] + 0.0501 * step
    assert Q.decide(Tt)
    # rotation: 0.05 pi/2 rad about any axis
    Q = O.RecombinePolicy(boot_frames=1)
    assert Q.decide(base)
    lim = 0.05 * math.pi / 2
    Tr = base.copy()
    Tr[:3, :3] = base[:3, :3] @ random_rotation_small(np.array([1.0, 2.0, 0.5]), 0.999 * lim)
    assert not Q.decide(Tr)
    Tr[:3, :3] = base[:3, :3] @ random_rotation_small(np.array([1.0, 2.0, 0.5]), 1.001 * lim)
    assert Q.decide(Tr)
    # the reference pose moves with every recombination
    T3 = Tr.copy()
    T3[:3, 3] += 0.03 * step
    assert not Q.decide(T3)
