"""Serving form: batched render and batched ICP give, per request, bitwise the result of the
same request served alone; the continuous-batching server agrees with the serial baseline."""
import math

import numpy as np
import pytest

import synth
from tests import parity as P

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dtsdf():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2301_12796_amd import dtsdf as lib
    return lib


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def tiny_map(dtsdf):
    gm = dtsdf.Map(P.tiny_gpu_params(dtsdf))
    for f in synth.tiny_frames(10):
        gm.integrate(_dev(f["depth"]), _dev(f["rgb"]), P.TINY_CAM, f["T_wc"])
    torch.cuda.synchronize()
    return gm


def _alloc(cam, dev="cuda"):
    H, W = cam.height, cam.width
    return dict(depth=torch.full((H, W), -7.0, device=dev),
                vertex=torch.full((3, H, W), -7.0, device=dev),
                normal=torch.full((3, H, W), -7.0, device=dev),
                rgba=torch.full((H, W, 4), 77, dtype=torch.uint8, device=dev),
                mask=torch.full((H, W), 77, dtype=torch.uint8, device=dev))


def test_render_batch_matches_single_renders(dtsdf, tiny_map):
    """Views of four sensors (320x240 .. 1280x720) and three pyramid levels in one launch."""
    sensors = synth.serving_sensors()
    views, singles = [], []
    for k, (cam, _) in enumerate(sensors):
        T = synth.tiny_render_pose(0.7 * k + 0.2)
        for l in range(3):
            c = dtsdf.level_camera(cam, l)
            out = _alloc(c)
            views.append((c, T, 0.2, 10.0, out))
            singles.append(tiny_map.render(c, T, 0.2, 10.0))
    print(f"case: render_batch of {len(views)} views", flush=True)
    tiny_map.render_batch(views)
    torch.cuda.synchronize()
    hits = 0
    for (c, _, _, _, out), ref in zip(views, singles):
        for key in ("depth", "vertex", "normal", "rgba", "mask"):
            assert torch.equal(out[key], ref[key]), key
        hits += int((ref["mask"] > 0).sum())
    assert hits > 10000


def test_ragged_views_single_equals_batch(dtsdf, tiny_map):
    """Views whose sizes are not whole tiles nor whole groups of the single-view launch's
    interleaved work tiles: every pixel written exactly once (the fill values never survive)
    and bitwise the batched launch's (plain 8x8 tiles)."""
    T = synth.tiny_render_pose(0.9)
    for W, H in ((1, 1), (7, 5), (203, 77), (9, 300), (161, 121)):
        f = 0.75 * max(W, H)
        cam = synth.scenes.Camera(W, H, f, f, (W - 1) / 2.0, (H - 1) / 2.0)
        print(f"case: ragged view {W}x{H}", flush=True)
        single = _alloc(cam)
        tiny_map.render(cam, T, 0.2, 10.0, out=single)
        batch = _alloc(cam)
        tiny_map.render_batch([(cam, T, 0.2, 10.0, batch)])
        torch.cuda.synchronize()
        assert not (single["mask"] == 77).any() and not (single["depth"] == -7.0).any()
        for key in ("depth", "vertex", "normal", "rgba", "mask"):
            assert torch.equal(single[key], batch[key]), (W, H, key)


def test_render_batch_of_one_and_empty(dtsdf, tiny_map):
    cam, _ = synth.serving_sensors()[1]
    T = synth.tiny_render_pose(1.1)
    out = _alloc(cam)
    tiny_map.render_batch([(cam, T, 0.2, 10.0, out)])
    ref = tiny_map.render(cam, T, 0.2, 10.0)
    for key in ("depth", "vertex", "normal", "rgba", "mask"):
        assert torch.equal(out[key], ref[key]), key
    tiny_map.render_batch([])            # no views: nothing to do, no error


def _live_levels(dtsdf, depth, cam):
    pyr = [depth]
    for _ in range(2):
        pyr.append(dtsdf.depth_downsample(pyr[-1]))
    return [dtsdf.vertex_normal(pyr[l], dtsdf.level_camera(cam, l)) for l in range(3)]


def test_icp_step_batch_matches_icp_step(dtsdf, tiny_map):
    """Three requests (SE(3) and Sim(3), different sensors) advanced together for six
    iterations; each pose and result equals the one icp_step gives for that request alone."""
    work = synth.serving_workload(3, seed=21, device="cuda")
    sensors = synth.serving_sensors()
    reqs, host_T, levels = [], [], []
    for k, w in enumerate(work):
        cam, _ = sensors[w["sensor"]]
        c = dtsdf.level_camera(cam, 1)
        m = tiny_map.render(c, w["T_model"], outputs=("vertex", "normal", "mask"))
        lv, ln = _live_levels(dtsdf, _dev(w["depth"]), cam)[1]
        dim = 6 if k == 0 else 7
        dT0 = w["dT0"].copy()
        if dim == 6:
            dT0[:3, :3] /= np.cbrt(np.linalg.det(dT0[:3, :3]))
        reqs.append(dtsdf.IcpRequest(lv, ln, c, m["vertex"], m["normal"], m["mask"], c,
                                     _dev(dT0), torch.ones(1, dtype=torch.int32, device="cuda"),
                                     torch.zeros(dtsdf.ICP_RESULT_BYTES, dtype=torch.uint8,
                                                 device="cuda"), dim=dim))
        host_T.append(dT0)
        levels.append((lv, ln, c, m))
    for it in range(6):
        print(f"case: icp_step_batch iteration {it}", flush=True)
        dtsdf.icp_step_batch(reqs)
        for k, q in enumerate(reqs):
            lv, ln, c, m = levels[k]
            status, T, res = dtsdf.icp_step(lv, ln, c, m["vertex"], m["normal"], m["mask"], c,
                                            host_T[k], dim=q.dim)
            assert status == dtsdf.OK
            host_T[k] = T
            got = q.pose.cpu().numpy()
            assert np.array_equal(got, T), (k, it, np.abs(got - T).max())
            r = dtsdf.decode_result(q.result)
            assert r["inliers"] == res["inliers"] and r["error"] == res["error"]
            assert r["step_norm"] == res["step_norm"]


def test_icp_step_batch_respects_inactive_flag(dtsdf, tiny_map):
    """A request whose device flag is 0 is left untouched; min_step clears the flag."""
    w = synth.serving_workload(1, seed=22, device="cuda")[0]
    cam, _ = synth.serving_sensors()[w["sensor"]]
    m = tiny_map.render(cam, w["T_model"], outputs=("vertex", "normal", "mask"))
    lv, ln = dtsdf.vertex_normal(_dev(w["depth"]), cam)
    pose = _dev(w["dT0"])
    active = torch.zeros(1, dtype=torch.int32, device="cuda")
    q = dtsdf.IcpRequest(lv, ln, cam, m["vertex"], m["normal"], m["mask"], cam, pose, active,
                         None, dim=7)
    dtsdf.icp_step_batch([q])
    assert np.array_equal(pose.cpu().numpy(), w["dT0"])
    active.fill_(1)
    q.min_step = 1e9                       # any step is below it: one step, then inactive
    dtsdf.icp_step_batch([q])
    assert int(active.item()) == 0
    after = pose.cpu().numpy()
    assert not np.array_equal(after, w["dT0"])
    dtsdf.icp_step_batch([q])
    assert np.array_equal(pose.cpu().numpy(), after)


def test_server_matches_serial_and_converges(dtsdf, tiny_map):
    """Twelve requests over four sensors served with three slots (so requests join and
    leave a running batch): final poses are bitwise those of the serial path, each
    registered frame fits the model to the depth noise, and the Sim(3) scale recovers the
    sensors' depth factors.  (The sphere leaves rotations about its centre, and a view of the
    plate alone leaves the scale, weakly constrained; a request can then settle elsewhere
    along that valley, so the scale is judged over the set of requests.)"""
    from paper_2301_12796_amd import serve
    sensors = synth.serving_sensors()
    work = synth.serving_workload(12, seed=23, device="cuda")

    def requests():
        return [serve.Request(k, w["arrival"], w["sensor"], _dev(w["depth"]), w["T_model"],
                              w["dT0"]) for k, w in enumerate(work)]
    srv = serve.Server(tiny_map, sensors, slots=3)
    print("case: server, 12 requests, 3 slots", flush=True)
    got = {r.rid: r for r in srv.run(requests(), realtime=False)}
    assert max(srv.batch_sizes) == 3 and len(got) == 12
    print("case: serial baseline, 12 requests", flush=True)
    ref = {r.rid: r for r in serve.serve_serial(tiny_map, sensors, requests(), realtime=False)}
    errs = []
    for k, w in enumerate(work):
        a, b = got[k].pose, ref[k].pose
        assert np.array_equal(a, b), (k, np.abs(a - b).max())
        assert got[k].error == ref[k].error and got[k].inliers == ref[k].inliers
        s = np.cbrt(np.linalg.det(a[:3, :3]))
        rms = math.sqrt(got[k].error / max(got[k].inliers, 1))
        errs.append(abs(math.log(s * w["scale"])))
        print(f"[serve {k}] sensor {w['sensor']} scale {s * w['scale']:.5f} "
              f"rms {rms * 1e3:.3f} mm inliers {got[k].inliers}", flush=True)
        assert rms < 2e-3 and got[k].inliers > 500
    errs = np.array(errs)
    assert np.median(errs) < 3e-3 and np.mean(errs < 5e-3) >= 0.75


def test_server_memory_budget_limits_admission(dtsdf, tiny_map):
    from paper_2301_12796_amd import serve
    sensors = synth.serving_sensors()
    work = synth.serving_workload(4, seed=24, device="cuda")
    big = max(serve.request_bytes(c) for c, _ in sensors)
    srv = serve.Server(tiny_map, sensors, slots=4, budget_bytes=big)
    reqs = [serve.Request(k, w["arrival"], w["sensor"], _dev(w["depth"]), w["T_model"],
                          w["dT0"]) for k, w in enumerate(work)]
    done = srv.run(reqs, realtime=False)
    assert len(done) == 4 and srv.peak_bytes <= big
    with pytest.raises(ValueError):
        serve.Server(tiny_map, sensors, slots=2, budget_bytes=big - 1)


def test_render_batch_room_views_match_single_renders(dtsdf):
    """Eight 640x480 views of a room map fused from 20 frames rendered in one persistent
    launch (the bench's batched form) equal the one-view launches bitwise."""
    cam = P.ROOM_CAM
    gm = dtsdf.Map(P.room_gpu_params(dtsdf))
    for f in synth.room_frames(range(0, 300, 15), device="cuda"):
        gm.integrate(_dev(f["depth"]), _dev(f["rgb"]), cam, f["T_wc"])
    poses = [synth.room_pose(k) for k in range(7, 300, 37)]
    outs = [_alloc(cam) for _ in poses]
    gm.render_batch([(cam, T, 0.2, 10.0, o) for T, o in zip(poses, outs)])
    hits = 0
    for T, o in zip(poses, outs):
        ref = P.to_numpy_out(gm.render(cam, T))
        got = P.to_numpy_out(o)
        for k in ("depth", "vertex", "normal", "rgba", "mask"):
            assert np.array_equal(got[k], ref[k]), k
        hits += int(ref["mask"].sum())
    print(f"case: batched room views, {len(poses)} views, {hits} hits", flush=True)
    assert hits > 0.9 * len(poses) * cam.width * cam.height


@pytest.mark.parametrize("dim,photo", [(6, False), (7, False), (6, True)])
def test_device_loop_icp_equals_host_loop(dtsdf, dim, photo):
    """icp_device (every iteration enqueued through icp_step_batch, pose and convergence flag
    on the device) gives bitwise the pose of the host loop icp(), on a preprocessed room
    frame, in SE(3), Sim(3) and combined with the photometric term."""
    sc = synth.room_scene()
    cam = P.ROOM_CAM
    T = synth.room_pose(70)
    s = 1.0 if dim == 6 else 1.03
    f = synth.render_frame(sc, cam, T, noise="quadratic", sigma=0.0012, seed=9, depth_scale=s,
                           texture_period=0.25)
    dT0 = synth.perturb_pose(0.02, math.radians(2.0), np.random.default_rng(11))
    levels, refs = [], []
    ri = dtsdf.intensity(_dev(synth.render_frame(sc, cam, T, texture_period=0.25)["rgb"]))
    for l in range(3):
        c = cam.level(l)
        g = synth.render_frame(sc, c, T)
        V = (c.pixel_rays() * g["true_depth"][..., None]).astype(np.float32)
        levels.append((_dev(V.transpose(2, 0, 1)), _dev(g["normal"].astype(np.float32).transpose(2, 0, 1)),
                       _dev(g["hit"].astype(np.uint8)), c))
        refs.append((ri, c))
        if l < 2:
            ri = dtsdf.intensity_downsample(ri)
    kw = dict(dim=dim, preprocess=dtsdf.Preprocess())
    if photo:
        kw.update(live_rgb=_dev(f["rgb"]), ref_levels=refs)
    T_host, log = dtsdf.icp(_dev(f["depth"]), cam, levels, dT0, **kw)
    T_dev = dtsdf.icp_device(_dev(f["depth"]), cam, levels, dT0, **kw)
    print(f"case: device-loop icp dim={dim} photo={photo}: {len(log)} host steps, "
          f"|t| {np.linalg.norm(T_dev[:3, 3]):.2e} m", flush=True)
    assert np.array_equal(T_host, T_dev)


def test_render_levels_equal_single_renders(dtsdf, tiny_map):
    """The model pyramid in one batched launch equals the three single renders bitwise."""
    cam = synth.scenes.Camera(320, 240, 240.0, 240.0, 159.5, 119.5)
    T = synth.tiny_render_pose(0.7)
    lv = dtsdf.render_levels(tiny_map, cam, T)
    for v, n, m, c in lv:
        ref = tiny_map.render(c, T, outputs=("vertex", "normal", "mask"))
        assert torch.equal(v, ref["vertex"]) and torch.equal(n, ref["normal"])
        assert torch.equal(m, ref["mask"])
    assert int(lv[0][2].sum()) > 1000
