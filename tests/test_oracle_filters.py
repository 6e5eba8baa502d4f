"""Pins of the oracle's input preprocessing (Sec. 7, Sec. 8 parameters) and post-fusion error.

* support filter: a constant image, a plane and a one-pixel-wide line are kept whole; single
  speckles, two-pixel blobs and pixels with one supporting neighbour are removed; the relative
  threshold is inclusive;
* bilateral depth: a constant image and a linear ramp are fixed points (the ramp by the
  symmetry of the weights), a step far above sigma_r keeps both levels, a hole neither
  spreads nor changes its neighbours, and with sigma_r -> inf the filter is the normalised
  truncated Gaussian (scipy.ndimage.correlate);
* bilateral normal: a constant field is a fixed point, a 90 degree crease keeps both faces,
  with sigma_r -> inf it is the renormalised Gaussian average, outputs are unit length;
* post-fusion MAE on a hand-computed example.
"""
import math

import numpy as np
import scipy.ndimage

import synth

from oracle import oracle as O


def _gauss(sigma, r):
    v, u = np.mgrid[-r:r + 1, -r:r + 1]
    return np.exp(-(u * u + v * v) / (2.0 * sigma * sigma))


def test_support_filter_keeps_planes_and_lines():
    D = np.full((20, 30), 1.5)
    assert np.array_equal(O.depth_support_filter(D), D)          # corners have 3 neighbours
    vv, uu = np.mgrid[0:20, 0:30]
    ramp = 1.0 + 0.002 * uu + 0.001 * vv
    assert np.array_equal(O.depth_support_filter(ramp), ramp)
    L = np.zeros((9, 9))
    L[4, :] = 2.0                                                  # each pixel: 2 neighbours
    out = O.depth_support_filter(L)
    assert np.array_equal(out[4, 1:-1], L[4, 1:-1])
    assert out[4, 0] == 0 and out[4, -1] == 0                      # line ends: 1 neighbour


def test_support_filter_removes_speckles_and_blobs():
    D = np.zeros((12, 12))
    D[2, 2] = 1.0                                                  # isolated
    D[6, 6] = D[6, 7] = 1.2                                        # two-pixel blob
    P = np.full((12, 12), 2.0)
    P[5, 5] = 2.5                                                  # outlier inside a plane
    assert not O.depth_support_filter(D).any()
    out = O.depth_support_filter(P)
    assert out[5, 5] == 0 and (out > 0).sum() == 143
    # inclusive relative threshold (dyadic values, so the boundary case is exact): neighbours
    # exactly 1/64 of the depth away support, just above do not
    T = np.zeros((3, 3))
    T[1, 1] = 2.0
    T[1, 0] = T[1, 2] = 2.0 + 2.0 / 64
    assert O.depth_support_filter(T, 1.0 / 64)[1, 1] == 2.0
    T[1, 2] = 2.0 + 2.0 / 64 + 2.0 ** -20
    assert O.depth_support_filter(T, 1.0 / 64)[1, 1] == 0.0


def test_bilateral_depth_fixed_points_and_edges():
    D = np.full((24, 24), 1.7)
    np.testing.assert_allclose(O.bilateral_depth(D), D, rtol=0, atol=1e-14)
    vv, uu = np.mgrid[0:24, 0:24]
    ramp = 1.0 + 0.004 * uu - 0.003 * vv
    out = O.bilateral_depth(ramp)
    np.testing.assert_allclose(out[5:-5, 5:-5], ramp[5:-5, 5:-5], rtol=0, atol=1e-13)
    step = np.where(uu < 12, 1.0, 2.0)
    np.testing.assert_allclose(O.bilateral_depth(step), step, rtol=0, atol=1e-14)
    hole = D.copy()
    hole[10:13, 10:13] = 0.0
    out = O.bilateral_depth(hole)
    assert np.all(out[10:13, 10:13] == 0)
    np.testing.assert_allclose(out[hole > 0], 1.7, rtol=0, atol=1e-14)


def test_bilateral_depth_without_range_term_is_gaussian_smoothing():
    rng = np.random.default_rng(3)
    D = 1.0 + rng.uniform(0, 0.5, (30, 40))
    k = _gauss(5.0, 5)
    ref = scipy.ndimage.correlate(D, k / k.sum(), mode="constant")
    out = O.bilateral_depth(D, sigma_r=1e9)
    np.testing.assert_allclose(out[5:-5, 5:-5], ref[5:-5, 5:-5], rtol=1e-12)


def test_bilateral_normal_preserves_creases():
    N = np.zeros((20, 20, 3))
    N[:, :10] = [1.0, 0.0, 0.0]
    N[:, 10:] = [0.0, 0.0, -1.0]
    out = O.bilateral_normal(N)
    np.testing.assert_allclose(out, N, rtol=0, atol=1e-12)
    c = np.zeros((12, 12, 3))
    c[...] = np.array([0.3, -0.4, -0.866]) / np.linalg.norm([0.3, -0.4, -0.866])
    c[3, 4] = 0.0
    out = O.bilateral_normal(c)
    np.testing.assert_allclose(out[c.any(-1)], c[c.any(-1)], rtol=0, atol=1e-14)
    assert not out[3, 4].any()


def test_bilateral_normal_without_range_term_is_gaussian_average():
    rng = np.random.default_rng(5)
    N = rng.normal(size=(25, 25, 3)) * 0.1 + np.array([0.0, 0.0, -1.0])
    N /= np.linalg.norm(N, axis=-1, keepdims=True)
    k = _gauss(2.5, 5)
    acc = np.stack([scipy.ndimage.correlate(N[..., i], k, mode="constant") for i in range(3)], -1)
    ref = acc / np.linalg.norm(acc, axis=-1, keepdims=True)
    out = O.bilateral_normal(N, sigma_r_deg=1e9)
    np.testing.assert_allclose(out[5:-5, 5:-5], ref[5:-5, 5:-5], rtol=0, atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(O.bilateral_normal(N), axis=-1), 1.0, atol=1e-12)


def test_post_fusion_mae_example():
    r = np.array([[1.0, 2.0, 0.0], [1.5, 0.0, 3.0]])
    m = np.array([[1.1, 1.8, 2.0], [0.0, 0.0, 2.7]])
    mae, n = O.post_fusion_mae(r, m)
    assert n == 3 and math.isclose(mae, (0.1 + 0.2 + 0.3) / 3, rel_tol=1e-12)


def _plane_frame(cam, z=0.5):
    depth = np.full((cam.height, cam.width), z, np.float32)
    rgb = np.zeros((cam.height, cam.width, 3), np.uint8)
    rgb[...] = (30, 140, 250)
    return depth, rgb


def test_fusion_with_its_own_normals_is_unchanged():
    """Caller normals equal to the cross-product normals reproduce the default fusion."""
    from synth.scenes import TINY_CAMERA as cam
    frames = synth.tiny_frames(3)
    a = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04))
    b = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04))
    for f in frames:
        a.integrate(f["depth"], f["rgb"], cam, f["T_wc"])
        _, N, _ = O.vertex_normal_map(f["depth"], cam)
        b.integrate(f["depth"], f["rgb"], cam, f["T_wc"], normals=N)
    ea, eb = a.export(), b.export()
    assert np.array_equal(ea["keys"], eb["keys"])
    assert np.array_equal(ea["sdf"], eb["sdf"]) and np.array_equal(ea["w"], eb["w"])


def test_fusion_with_given_normals_closed_form():
    """A frontal plane fused with the exact normal at every pixel (the image border
    included, where cross-product normals do not exist) stores the exact signed distance;
    normals on pixels without depth are ignored."""
    from synth.scenes import TINY_CAMERA as cam
    depth, rgb = _plane_frame(cam)
    N = np.zeros((cam.height, cam.width, 3))
    N[..., 2] = -1.0
    m = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04))
    m.integrate(depth, rgb, cam, np.eye(4), normals=N)
    b = m.export()
    from tests.test_oracle_pins import _voxel_positions
    x = _voxel_positions(b, 0.01)
    d_true = (0.5 - x[..., 2]) / O.f32(0.04)
    band = (b["w"] > 0) & (np.abs(d_true) <= 1)
    assert band.sum() > 10000
    assert np.max(np.abs(b["sdf"][band] - d_true[band])) < 1e-6
    # voxels seen by the border pixels are fused too (the default path has no normal there)
    ref = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04))
    ref.integrate(depth, rgb, cam, np.eye(4))
    assert (b["w"] > 0).sum() > (ref.export()["w"] > 0).sum()
    # normals where the depth is missing change nothing
    half = depth.copy()
    half[:, : cam.width // 2] = 0.0
    m1 = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04))
    m1.integrate(half, rgb, cam, np.eye(4), normals=N)
    N2 = N.copy()
    N2[:, : cam.width // 2] = 0.0
    m2 = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04))
    m2.integrate(half, rgb, cam, np.eye(4), normals=N2)
    e1, e2 = m1.export(), m2.export()
    assert np.array_equal(e1["keys"], e2["keys"]) and np.array_equal(e1["sdf"], e2["sdf"])
