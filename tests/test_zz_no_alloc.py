"""The allocation-free batched ICP entry point (icp_step_batch_iters_noalloc) against the
allocating one (icp_step_batch_iters) on the same requests, through the C ABI: two calls in
a row, the second with fewer requests on smaller images, each equal to the allocating call."""
import numpy as np
import pytest

import synth

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
    from tests import parity as P
    gm = dtsdf.Map(P.tiny_gpu_params(dtsdf))
    for f in synth.tiny_frames(10):
        gm.integrate(_dev(f["depth"]), _dev(f["rgb"]), P.TINY_CAM, f["T_wc"])
    torch.cuda.synchronize()
    return gm


def _requests(dtsdf, tiny_map, n, level, seed):
    """n registration requests (alternating SE(3) and Sim(3), four sensors) at pyramid
    level `level`, each with its own device pose, flag and result."""
    work = synth.serving_workload(n, seed=seed, device="cuda")
    sensors = synth.serving_sensors()
    reqs = []
    for k, w in enumerate(work):
        cam, _ = sensors[w["sensor"]]
        c = dtsdf.level_camera(cam, level)
        m = tiny_map.render(c, w["T_model"], outputs=("vertex", "normal", "mask"))
        d = _dev(w["depth"])
        for _ in range(level):
            d = dtsdf.depth_downsample(d)
        lv, ln = dtsdf.vertex_normal(d, c)
        dim = 6 if k % 2 == 0 else 7
        dT0 = w["dT0"].copy()
        if dim == 6:
            dT0[:3, :3] /= np.cbrt(np.linalg.det(dT0[:3, :3]))
        reqs.append(dtsdf.IcpRequest(lv, ln, c, m["vertex"], m["normal"], m["mask"], c,
                                     _dev(dT0), torch.ones(1, dtype=torch.int32, device="cuda"),
                                     torch.zeros(dtsdf.ICP_RESULT_BYTES, dtype=torch.uint8,
                                                 device="cuda"), dim=dim))
    return reqs


def _copy(dtsdf, q):
    return dtsdf.IcpRequest(q.live_vertex, q.live_normal, q.live_cam, q.model_vertex,
                            q.model_normal, q.model_mask, q.model_cam, q.pose.clone(),
                            q.active.clone(), q.result.clone(), dim=q.dim, params=q.params,
                            min_step=q.min_step)


def test_noalloc_equals_allocating_batch(dtsdf, tiny_map):
    cases = [(dtsdf.NOALLOC_MAX_REQUESTS, 1, 31, 4), (3, 2, 32, 6)]
    for n, level, seed, iters in cases:
        print(f"case: icp_step_batch_iters_noalloc n={n} level={level} iterations={iters}",
              flush=True)
        ref = _requests(dtsdf, tiny_map, n, level, seed)
        mine = [_copy(dtsdf, q) for q in ref]
        dtsdf.icp_step_batch_iters(ref, iters)
        dtsdf.icp_step_batch_iters_noalloc(mine, iters)
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(ref, mine)):
            pa, pb = a.pose.cpu().numpy(), b.pose.cpu().numpy()
            # the same kernels in the same order: equal to the allocating call
            assert np.array_equal(pa, pb), (n, k, np.abs(pa - pb).max())
            assert int(a.active.item()) == int(b.active.item())
            ra, rb = dtsdf.decode_result(a.result), dtsdf.decode_result(b.result)
            assert ra["inliers"] == rb["inliers"] and ra["error"] == rb["error"]
            assert ra["inliers"] > 0


def test_noalloc_rejects_oversized_batches(dtsdf, tiny_map):
    reqs = _requests(dtsdf, tiny_map, 1, 2, 33) * (dtsdf.NOALLOC_MAX_REQUESTS + 1)
    with pytest.raises(dtsdf.DtsdfError):
        dtsdf.icp_step_batch_iters_noalloc(reqs, 1)
    dtsdf.icp_step_batch_iters_noalloc([], 1)     # an empty batch is a no-op
