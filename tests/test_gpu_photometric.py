"""Parity of combined geometric + photometric ICP (icp_step_rgb, Sec. 5.2-5.3) with the FP64
oracle, through the C ABI: grey conversion and pyramid, normal equations of one step in the
frame-to-frame and keyframe forms, three-level convergence, and the textured plane whose
in-plane offset only the photometric term recovers."""
import math

import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import parity as P

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TEX = 0.25      # solid texture period [m]


@pytest.fixture(scope="module")
def dtsdf():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2301_12796_amd import dtsdf as lib
    return lib


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _analytic_model(sc, cam, T):
    f = synth.render_frame(sc, cam, T)
    V = cam.pixel_rays() * f["true_depth"][..., None]
    return V.astype(np.float32).astype(np.float64), \
        f["normal"].astype(np.float32).astype(np.float64), f["hit"].astype(np.uint8)


def _keyframe_offset():
    K = np.eye(4)
    K[:3, :3] = synth.scenes.random_rotation_small(np.array([0.3, 1.0, 0.2]), math.radians(2.0))
    K[:3, 3] = [-0.04, 0.02, 0.01]
    return K


def test_intensity_and_pyramid_match_oracle(dtsdf):
    f = synth.render_frame(synth.room_scene(), P.ROOM_CAM, synth.room_pose(20),
                           texture_period=TEX)
    g = dtsdf.intensity(_dev(f["rgb"]))
    ref = O.intensity_pyramid(O.intensity(f["rgb"]), 3)
    levels = [g, dtsdf.intensity_downsample(g)]
    levels.append(dtsdf.intensity_downsample(levels[1]))
    for l in range(3):
        assert np.max(np.abs(levels[l].cpu().numpy() - ref[l])) < 2e-6


@pytest.mark.parametrize("keyframe", [False, True])
@pytest.mark.parametrize("dim", [6, 7])
def test_icp_step_rgb_normal_equations(dtsdf, dim, keyframe):
    """One combined step: H, g, error, counts and the updated pose against the oracle's
    associate_reduce_rgb on the same float32 inputs."""
    sc = synth.room_scene()
    cam = P.ROOM_CAM
    T = synth.room_pose(40)
    fl = synth.render_frame(sc, cam, T, noise="quadratic", sigma=0.0012, seed=5,
                            texture_period=TEX)
    T_ref = T @ _keyframe_offset() if keyframe else T
    fr = synth.render_frame(sc, cam, T_ref, texture_period=TEX)
    T_rs = np.linalg.inv(T_ref) @ T
    V, N, M = _analytic_model(sc, cam, T)
    dT = synth.perturb_pose(0.01, math.radians(1.0), np.random.default_rng(7))
    lv, ln = dtsdf.vertex_normal(_dev(fl["depth"]), cam)
    li = dtsdf.intensity(_dev(fl["rgb"]))
    ri = dtsdf.intensity(_dev(fr["rgb"]))
    photo = dtsdf.Photo(li, ri, cam, T_rs, 0.1, 0.175)
    status, T_new, res = dtsdf.icp_step(lv, ln, cam, _dev(V.transpose(2, 0, 1).astype(np.float32)),
                                        _dev(N.transpose(2, 0, 1).astype(np.float32)), _dev(M),
                                        cam, dT, dim=dim, photo=photo)
    assert status == dtsdf.OK
    LV, LN, LOK = O.vertex_normal_map(fl["depth"], cam)
    Li = li.cpu().numpy().astype(np.float64)
    Ri = ri.cpu().numpy().astype(np.float64)
    Href, gref, err, cnt, cph = O.associate_reduce_rgb(LV, LN, LOK, Li, V, N, M, cam, Ri, cam,
                                                       T_rs, dT, dim, lam=0.1, max_err=0.175)
    print(f"[icp rgb dim={dim} kf={keyframe}] inliers {res['inliers']} / {cnt}, photometric "
          f"{res['photometric']} / {cph}", flush=True)
    assert abs(res["inliers"] - cnt) <= max(5, 1e-4 * cnt)
    assert abs(res["photometric"] - cph) <= max(5, 2e-4 * cph)
    assert cph > 100000
    np.testing.assert_allclose(res["H"], Href, rtol=2e-3, atol=1e-3 * np.abs(Href).max())
    np.testing.assert_allclose(res["g"], gref, rtol=5e-3, atol=2e-3 * np.abs(gref).max())
    T_ref_step = O.exp_map(O.solve_step(Href, gref)) @ dT
    assert np.max(np.abs(T_new - T_ref_step)) < 2e-5


@pytest.mark.parametrize("keyframe", [False, True])
def test_combined_icp_converges_like_oracle(dtsdf, keyframe):
    """Three levels (10/5/4 iterations), combined geometric + photometric: final poses agree
    within 2e-5 rad / 2e-5 m."""
    sc = synth.room_scene()
    cam = P.ROOM_CAM
    T = synth.room_pose(70)
    fl = synth.render_frame(sc, cam, T, noise="quadratic", sigma=0.0012, seed=9,
                            texture_period=TEX)
    T_ref = T @ _keyframe_offset() if keyframe else T
    fr = synth.render_frame(sc, cam, T_ref, texture_period=TEX)
    T_rs = np.linalg.inv(T_ref) @ T
    dT0 = synth.perturb_pose(0.02, math.radians(2.0), np.random.default_rng(11))
    levels_o, levels_g = [], []
    Iref_o = O.intensity_pyramid(O.intensity(fr["rgb"]), 3)
    ri = [dtsdf.intensity(_dev(fr["rgb"]))]
    for l in range(1, 3):
        ri.append(dtsdf.intensity_downsample(ri[-1]))
    ref_o, ref_g = [], []
    for l in range(3):
        c = cam.level(l)
        V, N, M = _analytic_model(sc, c, T)
        levels_o.append((V, N, M, c))
        levels_g.append((_dev(V.transpose(2, 0, 1).astype(np.float32)),
                         _dev(N.transpose(2, 0, 1).astype(np.float32)), _dev(M), c))
        ref_o.append((ri[l].cpu().numpy().astype(np.float64), c))
        ref_g.append((ri[l], c))
    T_o, _ = O.icp_rgb(fl["depth"], fl["rgb"], cam, levels_o, ref_o, T_rs, dT0)
    T_g, log = dtsdf.icp(_dev(fl["depth"]), cam, levels_g, dT0, live_rgb=_dev(fl["rgb"]),
                         ref_levels=ref_g, T_ref_model=T_rs)
    ang = P.rotation_angle(T_g[:3, :3] @ T_o[:3, :3].T)
    dt = np.linalg.norm(T_g[:3, 3] - T_o[:3, 3])
    print(f"[combined icp kf={keyframe}] rot {ang:.2e} rad trans {dt:.2e} m, "
          f"{len(log)} steps", flush=True)
    assert ang < 2e-5 and dt < 2e-5
    # and both sit near the true offset (the live frame was rendered at T: identity)
    assert np.linalg.norm(T_g[:3, 3]) < 2e-3


def test_textured_plane_needs_the_photometric_term(dtsdf):
    cam = synth.scenes.Camera(160, 120, 120.0, 120.0, 79.5, 59.5)
    room = synth.scenes.Room(np.array([-5.0, -5.0, -5.0]), np.array([5.0, 5.0, 1.0]),
                             np.tile(np.array([200, 180, 160], np.uint8), (6, 1)))
    sc = synth.scenes.Scene(spheres=[], boxes=[], room=room)
    T_model = synth.look_at((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), up=(0.0, 1.0, 0.0))
    D = np.eye(4)
    D[:3, :3] = synth.scenes.random_rotation_small(np.array([0.0, 0.0, 1.0]), math.radians(1.0))
    D[:3, 3] = [0.02, -0.015, 0.0]
    fm = synth.render_frame(sc, cam, T_model, texture_period=TEX)
    fl = synth.render_frame(sc, cam, T_model @ D, texture_period=TEX)
    levels, ref = [], []
    ri = [dtsdf.intensity(_dev(fm["rgb"]))]
    for l in range(1, 3):
        ri.append(dtsdf.intensity_downsample(ri[-1]))
    for l in range(3):
        c = cam.level(l)
        V, N, M = _analytic_model(sc, c, T_model)
        levels.append((_dev(V.transpose(2, 0, 1).astype(np.float32)),
                       _dev(N.transpose(2, 0, 1).astype(np.float32)), _dev(M), c))
        ref.append((ri[l], c))
    Tg, _ = dtsdf.icp(_dev(fl["depth"]), cam, levels, np.eye(4))
    assert np.linalg.norm(Tg[:3, 3] - D[:3, 3]) > 5e-3
    Tc, _ = dtsdf.icp(_dev(fl["depth"]), cam, levels, np.eye(4), live_rgb=_dev(fl["rgb"]),
                      ref_levels=ref)
    assert np.linalg.norm(Tc[:3, 3] - D[:3, 3]) < 1e-3
    assert P.rotation_angle(Tc[:3, :3].T @ D[:3, :3]) < math.radians(0.05)
