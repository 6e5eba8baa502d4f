"""Parity of brick recycling (dtsdf_recycle, Sec. 3) with the FP64 oracle, through the C ABI.

Workload: a scene with a ball fused from 4 views, then 10 views of the scene without it
(carving weight 1), so that carving turns the ball's bricks into free space; recycling at
t_free = 0.5.  Checked: the same bricks are recycled on both sides (bricks whose decision sits
within 1e-4 of t_free, or that hold a voxel the oracle flags as borderline, are skipped), the
recycled maps agree voxel-wise, the recycled map renders bitwise like a fresh map holding the
same bricks (the render index is rebuilt from a cleared grid), and fusing the ball again
reuses freed bricks (reset to an unused brick's state) with the maps still in agreement."""
import numpy as np
import pytest

import synth
from synth.scenes import look_at, render_frame
from oracle import oracle as O
from tests import parity as P
from tests.test_oracle_recycle import _scenes, carving_workload

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

T_FREE = 0.5


@pytest.fixture(scope="module")
def dtsdf():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2301_12796_amd import dtsdf as lib
    return lib


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _params(dtsdf):
    return dtsdf.Params(voxel_size=0.01, truncation=0.04, w_carve=1.0, brick_capacity=1 << 16,
                        hash_buckets=1 << 16)


def _decisions(blob, t_free):
    """Per brick: recycled by the definition, and whether the decision is borderline."""
    obs = blob["w"] > 0
    mn = np.where(obs, blob["sdf"], np.inf).min(1)
    free = mn >= np.float32(t_free)
    border = (np.abs(mn - t_free) < 1e-4) | blob["border"].astype(bool).any(1) | \
        (obs & (blob["w"] < 1e-5)).any(1)
    return free, border


def test_recycle_matches_oracle(dtsdf):
    cam, frames = carving_workload()
    gm = dtsdf.Map(_params(dtsdf))
    om = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04, w_carve=1.0))
    for f in frames:
        gm.integrate(_dev(f["depth"]), _dev(f["rgb"]), cam, f["T_wc"])
        om.integrate(f["depth"], f["rgb"], cam, f["T_wc"])
    gb0, ob0 = gm.export(), om.export()
    assert P.compare_maps(gb0, ob0, n_frames=len(frames), name="before recycling")["ok"]
    free_o, border_o = _decisions(ob0, T_FREE)
    n_g = gm.recycle(T_FREE)
    n_o = om.recycle(T_FREE)
    gb1, ob1 = gm.export(), om.export()
    gset0, gset1 = set(map(tuple, gb0["keys"])), set(map(tuple, gb1["keys"]))
    oidx = {tuple(k): i for i, k in enumerate(ob0["keys"])}
    checked = mism = 0
    for k in gset0 & set(oidx):
        i = oidx[k]
        if border_o[i]:
            continue
        checked += 1
        mism += (k not in gset1) != bool(free_o[i])
    print(f"case: recycle t_free={T_FREE}: gpu {n_g}, oracle {n_o}, checked {checked}, "
          f"mismatches {mism}", flush=True)
    assert n_o > 50 and mism == 0 and abs(n_g - n_o) <= max(3, 0.02 * n_o)
    assert gm.info()["bricks"] == len(gb1["keys"]) == len(gb0["keys"]) - n_g
    assert P.compare_maps(gb1, ob1, n_frames=len(frames), name="after recycling")["ok"]

    # the recycled map renders exactly like a fresh map holding the same bricks
    fresh = dtsdf.Map(_params(dtsdf))
    fresh.load(gb1)
    for T in (look_at((0.9, -0.4, 0.1), (0.0, 0.0, 0.0)), synth.tiny_render_pose(1.3)):
        a = P.to_numpy_out(gm.render(cam, T))
        b = P.to_numpy_out(fresh.render(cam, T))
        for key in ("depth", "normal", "rgba", "mask"):
            assert np.array_equal(a[key], b[key]), key

    # the ball returns: new bricks come from the free list, reset to an unused brick's state
    with_ball = _scenes()[0]
    more = []
    for k, T in enumerate(synth.tiny_cameras(3, seed=9)):
        f = render_frame(with_ball, cam, T, noise="const", sigma=0.0005, seed=900 + k,
                         z_max=10.0)
        gm.integrate(_dev(f["depth"]), _dev(f["rgb"]), cam, T)
        om.integrate(f["depth"], f["rgb"], cam, T)
        more.append(f)
    gb2, ob2 = gm.export(), om.export()
    grown = len(gb2["keys"]) - len(gb1["keys"])
    print(f"case: refuse after recycling: {grown} bricks back", flush=True)
    assert grown > 0.5 * n_g
    assert gm.info()["bricks"] == len(gb2["keys"])
    assert P.compare_maps(gb2, ob2, n_frames=len(frames) + len(more), name="refused")["ok"]


def test_recycle_rejects_dense_maps_and_bad_thresholds(dtsdf):
    dense = dtsdf.Map(P.tiny_gpu_params(dtsdf))
    with pytest.raises(dtsdf.DtsdfError):
        dense.recycle(0.5)
    sparse = dtsdf.Map(_params(dtsdf))
    with pytest.raises(dtsdf.DtsdfError):
        sparse.recycle(0.0)
    assert sparse.recycle(0.5) == 0
