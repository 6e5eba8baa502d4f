"""Precision form: float16 / int16 distances with uint8 weights, compensated float32 ICP.

Parity: the GPU and the oracle store the same codes (the oracle rounds its float64 running
averages with the same round-half-even rules), and render identical imported precision maps
identically.  Accuracy: the precision-form map fused on the GPU is rendered and compared with
the plain FP64 oracle, and the error is reported for depth, normal, colour and pose."""
import math

import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import parity as P

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

FORMATS = [(1, "f16"), (2, "i16")]


@pytest.fixture(scope="module")
def dtsdf():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2301_12796_amd import dtsdf as lib
    return lib


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _gpu_params(dtsdf, fmt, **kw):
    return P.tiny_gpu_params(dtsdf, sdf_fmt=fmt, w_fmt=dtsdf.W_U8, **kw)


@pytest.mark.parametrize("fmt,name", FORMATS)
def test_precision_integrate_codes_match(dtsdf, fmt, name):
    frames = synth.tiny_frames(10)
    om = O.OracleMap(P.tiny_oracle_params(sdf_fmt=fmt, w_fmt=1))
    gm = dtsdf.Map(_gpu_params(dtsdf, fmt))
    print(f"case: precision integrate {name}", flush=True)
    for f in frames:
        om.integrate(f["depth"], f["rgb"], P.TINY_CAM, f["T_wc"])
        gm.integrate(_dev(f["depth"]), _dev(f["rgb"]), P.TINY_CAM, f["T_wc"])
    g, o = gm.export(), om.export()
    assert np.array_equal(g["keys"], o["keys"])
    keep = o["border"] == 0
    ds = np.abs(g["sdf"] - o["sdf"])[keep]
    dw = np.abs(g["w"] - o["w"])[keep]
    # one step of the square-law weight code (w = q^2 / 1024) at the larger weight
    wstep = (2.0 * np.sqrt(1024.0 * np.maximum(g["w"], o["w"])[keep]) + 1.0) / 1024.0
    quantum = 2.0 ** -10 if fmt == 1 else 1.0 / 32767.0
    exact = (ds == 0) & (dw == 0)
    print(f"[precision codes {name}] voxels {keep.sum()} exact {exact.mean():.6f} "
          f"max dsdf {ds.max():.3g} max dw {dw.max():.3g}", flush=True)
    assert exact.mean() > 0.9999
    assert ds.max() <= quantum and np.all(dw <= wstep)
    dc = np.abs(g["rgb"].astype(int) - o["rgb"].astype(int))[keep]
    assert dc.max() <= 1


@pytest.mark.parametrize("fmt,name", FORMATS)
def test_precision_render_identical_map(dtsdf, fmt, name):
    frames = synth.tiny_frames(10)
    om = O.OracleMap(P.tiny_oracle_params(sdf_fmt=fmt, w_fmt=1))
    for f in frames:
        om.integrate(f["depth"], f["rgb"], P.TINY_CAM, f["T_wc"])
    blob = om.export()
    gm = dtsdf.Map(_gpu_params(dtsdf, fmt))
    gm.load(blob)
    back = gm.export()                      # import/export of codes is lossless
    assert np.array_equal(back["sdf"], blob["sdf"]) and np.array_equal(back["w"], blob["w"])
    ref_map = O.OracleMap(P.tiny_oracle_params(sdf_fmt=fmt, w_fmt=1))
    ref_map.load(blob)
    for phi in (0.3, 2.9):
        T = synth.tiny_render_pose(phi)
        out = P.to_numpy_out(gm.render(P.TINY_CAM, T, z_far=2.5))
        ref = ref_map.render(P.TINY_CAM, T, z_far=2.5)
        P.compare_render(out, ref, name=f"precision {name} phi={phi}",
                         roots=(ref_map, P.TINY_CAM, T))


@pytest.mark.parametrize("fmt,name", FORMATS)
def test_precision_error_vs_fp64_oracle(dtsdf, fmt, name):
    """Accuracy of the precision form against the plain FP64 oracle (reported)."""
    frames = synth.tiny_frames(10)
    om = O.OracleMap(P.tiny_oracle_params())
    gq = dtsdf.Map(_gpu_params(dtsdf, fmt))
    for f in frames:
        om.integrate(f["depth"], f["rgb"], P.TINY_CAM, f["T_wc"])
        gq.integrate(_dev(f["depth"]), _dev(f["rgb"]), P.TINY_CAM, f["T_wc"])
    T = synth.tiny_render_pose()
    out = P.to_numpy_out(gq.render(P.TINY_CAM, T, z_far=2.5))
    ref = om.render(P.TINY_CAM, T, z_far=2.5)
    m = (out["mask"].ravel() > 0) & (ref.mask > 0)
    dz = np.abs(out["depth"].ravel()[m] - ref.depth[m])
    gn = out["normal"].reshape(3, -1).T[m]
    ang = np.degrees(np.arccos(np.clip((gn * ref.normal[m]).sum(1), -1, 1)))
    dc = np.abs(out["rgba"].reshape(-1, 4)[m, :3].astype(int) - ref.rgba[m, :3].astype(int))
    mism = int(((out["mask"].ravel() > 0) != (ref.mask > 0)).sum())
    print(f"[precision error {name}] hits {m.sum()} mask mismatch {mism} depth median "
          f"{np.median(dz):.2e} p99 {np.percentile(dz, 99):.2e} m, normal median "
          f"{np.median(ang):.3f} p99 {np.percentile(ang, 99):.3f} deg, colour median "
          f"{np.median(dc):.1f} p99 {np.percentile(dc, 99):.1f}", flush=True)
    assert np.median(dz) < 2e-4 and np.median(ang) < 1.0 and mism < 0.02 * m.sum()


def test_sim3_scaled_sensor_on_precision_map(dtsdf):
    """Second sensor with depth scaled by s ~ U[0.9, 1.1] registered in Sim(3) against views
    rendered from the precision (float16) map, with the compensated reduction; the oracle
    runs the same registration on the same rendered model maps."""
    s = synth.precision_scale()
    cam = P.ROOM_CAM
    sc = synth.tiny_scene()
    frames = synth.tiny_frames(10)
    gq = dtsdf.Map(_gpu_params(dtsdf, 1))
    for f in frames:
        gq.integrate(_dev(f["depth"]), _dev(f["rgb"]), P.TINY_CAM, f["T_wc"])
    T = synth.tiny_render_pose(0.9)
    live = synth.render_frame(sc, cam, T, noise="const", sigma=0.0005, seed=77,
                              depth_scale=s)["depth"]
    rng = np.random.default_rng(11)
    dT0 = synth.perturb_pose(0.01, math.radians(1.0), rng)
    dT0[:3, :3] *= 1.01 / s
    levels_g, levels_o = [], []
    for l in range(3):
        c = dtsdf.level_camera(cam, l)
        o = gq.render(c, T, z_far=2.5, outputs=("vertex", "normal", "mask"))
        levels_g.append((o["vertex"], o["normal"], o["mask"], c))
        V = o["vertex"].cpu().numpy().transpose(1, 2, 0).astype(np.float64)
        N = o["normal"].cpu().numpy().transpose(1, 2, 0).astype(np.float64)
        levels_o.append((V, N, o["mask"].cpu().numpy(), cam.level(l)))
    prm = dtsdf.IcpParams(compensated=True)
    T_g, _ = dtsdf.icp(_dev(live), cam, levels_g, dT0, dim=7, params=prm)
    T_o, _ = O.icp(live, cam, levels_o, dT0, dim=7)
    sg = np.cbrt(np.linalg.det(T_g[:3, :3]))
    so = np.cbrt(np.linalg.det(T_o[:3, :3]))
    dR = (T_g[:3, :3] / sg) @ np.linalg.inv(T_o[:3, :3] / so)
    ang = P.rotation_angle(dR)
    dt = np.linalg.norm(T_g[:3, 3] - T_o[:3, 3])
    print(f"[sim3 precision] scale gpu {sg:.7f} oracle {so:.7f} truth {1 / s:.7f}; "
          f"rot {ang:.2e} rad, trans {dt:.2e} m", flush=True)
    assert ang < 1e-5 and dt < 1e-5 and abs(sg - so) < 1e-5
    assert abs(sg - 1 / s) < 5e-3
