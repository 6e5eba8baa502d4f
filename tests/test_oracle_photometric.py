"""Pins of the oracle's photometric terms of combined ICP (Sec. 5.2, Sec. 5.3).

* the Jacobian is checked against central finite differences of the residual itself, on an
  affine grey image (bilinear interpolation and central differences are exact there), for
  SE(3) and Sim(3) and a keyframe offset T_RS that is not the identity;
* a frontal textured plane fixes only depth and the two tilts geometrically: point-to-plane
  ICP cannot recover an in-plane offset, combined ICP does, against the frame rendered at
  the model pose (frame-to-frame) and against a keyframe rendered elsewhere (T_RS != I).
"""
import math

import numpy as np
import pytest

from synth.scenes import Camera, Scene, look_at, random_rotation_small, render_frame
from synth.scenes import Room
from oracle import oracle as O


def _affine_image(W=64, H=48):
    vv, uu = np.mgrid[0:H, 0:W].astype(np.float64)
    return 0.3 + 0.004 * uu - 0.003 * vv


def _pose(rng, t, a):
    T = np.eye(4)
    T[:3, :3] = random_rotation_small(rng.normal(size=3), a)
    T[:3, 3] = rng.normal(size=3) * t
    return T


@pytest.mark.parametrize("dim", [6, 7])
def test_photometric_jacobian_matches_finite_differences(dim):
    rng = np.random.default_rng(4)
    I_ref = _affine_image()
    cam = Camera(64, 48, 50.0, 50.0, 31.5, 23.5)
    T_rs = _pose(rng, 0.02, 0.05)
    dT = _pose(rng, 0.01, 0.03)
    n = 200
    P = np.stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.2, 0.2, n), rng.uniform(0.9, 1.3, n)], 1)
    I_live = rng.uniform(0.2, 0.8, n)
    J, r, ok = O.photometric_terms(P, I_live, I_ref, cam, T_rs, dT, dim, max_err=np.inf)
    assert ok.sum() > 150
    h = 1e-6
    num = np.zeros_like(J)
    for k in range(dim):
        e = np.zeros(dim)
        e[k] = h
        _, rp, okp = O.photometric_terms(P, I_live, I_ref, cam, T_rs, O.exp_map(e) @ dT, dim, np.inf)
        _, rm, okm = O.photometric_terms(P, I_live, I_ref, cam, T_rs, O.exp_map(-e) @ dT, dim, np.inf)
        assert np.array_equal(okp, ok) and np.array_equal(okm, ok)
        num[:, k] = (rp - rm) / (2 * h)
    assert np.max(np.abs(num - J)) < 1e-6 * max(1.0, np.max(np.abs(J)))


def _textured_plane_frames(T_model, T_live, T_kf, cam, period=0.25):
    """A textured wall at z = 1.0 facing the cameras (a room's far wall)."""
    room = Room(np.array([-5.0, -5.0, -5.0]), np.array([5.0, 5.0, 1.0]),
                np.tile(np.array([200, 180, 160], np.uint8), (6, 1)))
    sc = Scene(spheres=[], boxes=[], room=room)
    fm = render_frame(sc, cam, T_model, texture_period=period)
    fl = render_frame(sc, cam, T_live, texture_period=period)
    fk = render_frame(sc, cam, T_kf, texture_period=period)
    return fm, fl, fk


def _model_levels(f, cam, L=3):
    out = []
    for l in range(L):
        c = cam.level(l)
        s = 2 ** l
        z = f["true_depth"][::s, ::s][:c.height, :c.width]
        rays = c.pixel_rays()
        V = rays * z[..., None]
        N = f["normal"][::s, ::s][:c.height, :c.width]
        out.append((V, N, (z > 0).astype(np.uint8), c))
    return out


def _ref_levels(f, cam, L=3):
    I = O.intensity_pyramid(O.intensity(f["rgb"]), L)
    return [(I[l], cam.level(l)) for l in range(L)]


def _offset():
    D = np.eye(4)
    D[:3, :3] = random_rotation_small(np.array([0.0, 0.0, 1.0]), math.radians(1.0))
    D[:3, 3] = [0.02, -0.015, 0.0]
    return D


def test_textured_plane_is_recovered_only_with_the_photometric_term():
    cam = Camera(160, 120, 120.0, 120.0, 79.5, 59.5)
    T_model = look_at((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), up=(0.0, 1.0, 0.0))
    D = _offset()
    T_live = T_model @ D                      # live -> model transform is D
    fm, fl, _ = _textured_plane_frames(T_model, T_live, T_model, cam)
    levels = _model_levels(fm, cam)
    # geometric ICP: the in-plane offset is unobservable
    try:
        Tg, _ = O.icp(fl["depth"], cam, levels, np.eye(4))
        geo_err = np.linalg.norm(Tg[:3, 3] - D[:3, 3])
    except np.linalg.LinAlgError:
        geo_err = np.inf
    assert geo_err > 5e-3
    # combined ICP against the frame at the model pose (frame-to-frame, T_RS = I)
    Tc, log = O.icp_rgb(fl["depth"], fl["rgb"], cam, levels, _ref_levels(fm, cam), np.eye(4),
                        np.eye(4))
    assert np.linalg.norm(Tc[:3, 3] - D[:3, 3]) < 1e-3
    assert O.rotation_angle(Tc[:3, :3].T @ D[:3, :3]) < math.radians(0.05)
    assert all(e.get("photometric", 0) > 500 for e in log if "status" not in e)


def test_keyframe_offset_is_applied():
    """The reference image is a keyframe rendered 4 cm / 2 degrees away from the model pose;
    with T_RS = T_kf^-1 T_model combined ICP recovers the live offset, with T_RS = I it
    does not."""
    cam = Camera(160, 120, 120.0, 120.0, 79.5, 59.5)
    T_model = look_at((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), up=(0.0, 1.0, 0.0))
    K = np.eye(4)
    K[:3, :3] = random_rotation_small(np.array([0.3, 1.0, 0.2]), math.radians(2.0))
    K[:3, 3] = [-0.04, 0.02, 0.01]
    T_kf = T_model @ K
    D = _offset()
    T_live = T_model @ D
    fm, fl, fk = _textured_plane_frames(T_model, T_live, T_kf, cam)
    levels = _model_levels(fm, cam)
    T_rs = np.linalg.inv(T_kf) @ T_model
    Tc, _ = O.icp_rgb(fl["depth"], fl["rgb"], cam, levels, _ref_levels(fk, cam), T_rs, np.eye(4))
    assert np.linalg.norm(Tc[:3, 3] - D[:3, 3]) < 1e-3
    Tw, _ = O.icp_rgb(fl["depth"], fl["rgb"], cam, levels, _ref_levels(fk, cam), np.eye(4),
                      np.eye(4))
    assert np.linalg.norm(Tw[:3, 3] - D[:3, 3]) > 5e-3


def test_intensity_and_pyramid():
    rgb = np.zeros((4, 4, 3), np.uint8)
    rgb[..., 0] = 255
    assert np.allclose(O.intensity(rgb), 0.299)
    rgb[...] = 255
    assert np.allclose(O.intensity(rgb), 1.0)
    I = np.arange(16, dtype=np.float64).reshape(4, 4)
    p = O.intensity_pyramid(I, 2)
    assert np.allclose(p[1], [[2.5, 4.5], [10.5, 12.5]])
