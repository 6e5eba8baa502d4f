"""Parity of the view-dependent combined TSDF (dtsdf_volume_create / dtsdf_combine and the
render of a volume) with the FP64 oracle, through the C ABI (Sec. 4)."""
import math

import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import parity as P

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

# combined values: float32 weights from float32 central differences against float64; the
# value is a convex combination of stored values with relative weight errors ~1e-6
SDF_TOL = 2e-5


@pytest.fixture(scope="module")
def dtsdf():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2301_12796_amd import dtsdf as lib
    return lib


@pytest.fixture(scope="module")
def tiny_blobs():
    """Oracle maps of the tiny scene after 5 and after 10 frames (exported)."""
    m = O.OracleMap(P.tiny_oracle_params())
    frames = synth.tiny_frames(10)
    out = []
    for i, f in enumerate(frames):
        m.integrate(f["depth"], f["rgb"], P.TINY_CAM, f["T_wc"])
        if i in (4, 9):
            out.append(m.export())
    return out


@pytest.fixture(scope="module")
def room_blob():
    sc = synth.room_scene()
    m = O.OracleMap(P.room_oracle_params())
    for f in synth.room_frames([0, 100, 200], scene=sc):
        m.integrate(f["depth"], f["rgb"], P.ROOM_CAM, f["T_wc"])
    return m.export()


def _oracle_volume(params_fn):
    return O.OracleMap(params_fn(single_direction=True))



def compare_volumes(gpu: dict, orc: dict, name=""):
    """Voxel-wise comparison of a GPU volume export with the oracle's; voxels the oracle
    flags (frustum bound within 1e-6 px, fragile combination branch) are skipped."""
    gk = {tuple(k): i for i, k in enumerate(gpu["keys"])}
    ok = {tuple(k): i for i, k in enumerate(orc["keys"])}
    only_gpu, only_orc = len(set(gk) - set(ok)), len(set(ok) - set(gk))
    # plain integers in the assertion: pytest's explanation of a failing comparison of two
    # large sets diffs their full listings and can take minutes
    assert only_gpu == 0 and only_orc == 0, f"key sets differ: {only_gpu} GPU-only, {only_orc} oracle-only"
    keys = sorted(ok)
    gi = np.array([gk[k] for k in keys])
    oi = np.array([ok[k] for k in keys])
    keep = orc["border"][oi] == 0
    gw, ow = gpu["w"][gi][keep], orc["w"][oi][keep]
    st = dict(voxels=int(keep.size), flagged=int((~keep).sum()), valued=int((ow > 0).sum()),
              w_mismatch=int((gw != ow).sum()))
    both = (gw > 0) & (ow > 0)
    ds = np.abs(gpu["sdf"][gi][keep][both] - orc["sdf"][oi][keep][both])
    st["sdf_max"] = float(ds.max()) if ds.size else 0.0
    gwc, owc = gpu["wc"][gi][keep], orc["wc"][oi][keep]
    st["wc_mismatch"] = int((gwc != owc).sum())
    cb = (gwc > 0) & (owc > 0)
    dc = np.abs(gpu["rgb"][gi][keep][cb].astype(int) - orc["rgb"][oi][keep][cb].astype(int))
    st["rgb_max"] = int(dc.max()) if dc.size else 0
    print(f"[volume parity {name}] {st}", flush=True)
    assert st["w_mismatch"] == 0 and st["wc_mismatch"] == 0, st
    assert st["sdf_max"] <= SDF_TOL, st
    assert st["rgb_max"] <= P.COLOR_TOL, st
    return st


def test_combine_tiny_voxelwise(dtsdf, tiny_blobs):
    blob = tiny_blobs[1]
    gm = dtsdf.Map(P.tiny_gpu_params(dtsdf))
    gm.load(blob)
    src = O.OracleMap(P.tiny_oracle_params())
    src.load(blob)
    for phi in (0.3, 2.2):
        T = synth.tiny_render_pose(phi)
        print(f"case: tiny combine phi={phi}", flush=True)
        vol = dtsdf.Volume(gm, brick_capacity=1024, hash_buckets=1 << 12)
        vol.combine(gm, P.TINY_CAM, T)
        ref = _oracle_volume(P.tiny_oracle_params)
        ref.combine(src, P.TINY_CAM, T)
        st = compare_volumes(vol.export(), ref.export(), name=f"tiny phi={phi}")
        assert st["valued"] > 20000


def test_recombine_replaces_the_previous_volume(dtsdf, tiny_blobs):
    """A second full combination at another pose leaves no value outside its frustum."""
    blob = tiny_blobs[1]
    gm = dtsdf.Map(P.tiny_gpu_params(dtsdf))
    gm.load(blob)
    src = O.OracleMap(P.tiny_oracle_params())
    src.load(blob)
    cam = synth.scenes.Camera(80, 60, 120.0, 120.0, 39.5, 29.5)   # narrow view
    T1, T2 = synth.tiny_render_pose(0.3), synth.tiny_render_pose(1.9)
    vol = dtsdf.Volume(gm, brick_capacity=1024, hash_buckets=1 << 12)
    vol.combine(gm, cam, T1)
    vol.combine(gm, cam, T2)
    ref = _oracle_volume(P.tiny_oracle_params)
    ref.combine(src, cam, T2)
    compare_volumes(vol.export(), ref.export(), name="tiny recombined")


def test_fill_tiny_voxelwise(dtsdf, tiny_blobs):
    """Combine after 5 frames, then the map gains 5 more frames and the voxels without a
    value inside the next frame's frustum are filled for the first combination's centre."""
    gm = dtsdf.Map(P.tiny_gpu_params(dtsdf))
    src = O.OracleMap(P.tiny_oracle_params())
    T1, T2 = synth.tiny_render_pose(0.3), synth.tiny_render_pose(0.45)
    vol = dtsdf.Volume(gm, brick_capacity=1024, hash_buckets=1 << 12)
    ref = _oracle_volume(P.tiny_oracle_params)
    gm.load(tiny_blobs[0])
    src.load(tiny_blobs[0])
    vol.combine(gm, P.TINY_CAM, T1)
    ref.combine(src, P.TINY_CAM, T1)
    before = ref.export()
    src2 = O.OracleMap(P.tiny_oracle_params())
    src2.load(tiny_blobs[1])
    gm.load(tiny_blobs[1])
    print("case: tiny fill", flush=True)
    vol.combine(gm, P.TINY_CAM, T1, T_frustum=T2, margin=0.0, only_missing=True)
    ref.combine(src2, P.TINY_CAM, T1, T_frustum=T2, margin=0.0, only_missing=True)
    after = ref.export()
    assert (after["w"] > 0).sum() > (before["w"] > 0).sum()
    compare_volumes(vol.export(), after, name="tiny fill")


def test_render_volume_tiny_identical(dtsdf, tiny_blobs):
    """The oracle's combined volume imported into a GPU volume: renders agree at the
    direct path's bars (same lattice, hit test and refinement)."""
    src = O.OracleMap(P.tiny_oracle_params())
    src.load(tiny_blobs[1])
    gm = dtsdf.Map(P.tiny_gpu_params(dtsdf))
    for phi in (0.3, 2.2, 4.0):
        T = synth.tiny_render_pose(phi)
        ref = _oracle_volume(P.tiny_oracle_params)
        ref.combine(src, P.TINY_CAM, T)
        rb = ref.export()
        vol = dtsdf.Volume(gm, brick_capacity=1024, hash_buckets=1 << 12)
        vol.load(rb)
        rr = _oracle_volume(P.tiny_oracle_params)
        rr.load(rb)
        print(f"case: tiny volume render phi={phi}", flush=True)
        out = P.to_numpy_out(vol.render(P.TINY_CAM, T, z_far=2.5))
        st = P.compare_render(out, rr.render(P.TINY_CAM, T, z_far=2.5), name=f"volume phi={phi}",
                              roots=(rr, P.TINY_CAM, T))
        assert st["compared"] > 3000


def test_render_volume_room_sampled(dtsdf, room_blob):
    """Room map (3 frames, 640x480, 5 mm): the oracle's combined volume for pose 37 imported
    into a GPU volume and rendered in the benchmark's launch configuration; the oracle renders
    3000 sampled pixels plus two full rows."""
    src = O.OracleMap(P.room_oracle_params())
    src.load(room_blob)
    T = synth.room_pose(37)
    ref = _oracle_volume(P.room_oracle_params)
    ref.combine(src, P.ROOM_CAM, T)
    rb = ref.export()
    gm = dtsdf.Map(P.room_gpu_params(dtsdf))
    vol = dtsdf.Volume(gm, brick_capacity=1 << 17, hash_buckets=1 << 18)
    vol.load(rb)
    rr = _oracle_volume(P.room_oracle_params)
    rr.load(rb)
    print("case: room volume render pose 37", flush=True)
    out = P.to_numpy_out(vol.render(P.ROOM_CAM, T))
    pix = P.random_pixels(P.ROOM_CAM, 3000, seed=37)
    rows = np.stack(np.meshgrid(np.arange(640), [100, 333]), -1).reshape(-1, 2)
    pix = np.concatenate([pix, rows])
    st = P.compare_render(out, rr.render(P.ROOM_CAM, T, pixels=pix), pixels=pix,
                          name="room volume", roots=(rr, P.ROOM_CAM, T))
    assert st["hits"] > 1000


def test_combine_and_render_room(dtsdf, room_blob):
    """Room map (3 frames, 640x480, 5 mm): combine voxel-wise, then the oracle's volume
    rendered on the GPU at sampled pixels, in the benchmark's launch configuration."""
    gm = dtsdf.Map(P.room_gpu_params(dtsdf))
    gm.load(room_blob)
    src = O.OracleMap(P.room_oracle_params())
    src.load(room_blob)
    T = synth.room_pose(37)
    print("case: room combine pose 37", flush=True)
    vol = dtsdf.Volume(gm, brick_capacity=1 << 17, hash_buckets=1 << 18)
    vol.combine(gm, P.ROOM_CAM, T)
    ref = _oracle_volume(P.room_oracle_params)
    ref.combine(src, P.ROOM_CAM, T)
    rb = ref.export()
    st = compare_volumes(vol.export(), rb, name="room pose 37")
    assert st["valued"] > 1_000_000
    print("case: room volume render pose 37", flush=True)
    vol.load(rb)
    rr = _oracle_volume(P.room_oracle_params)
    rr.load(rb)
    out = P.to_numpy_out(vol.render(P.ROOM_CAM, T))
    pix = P.random_pixels(P.ROOM_CAM, 3000, seed=37)
    rows = np.stack(np.meshgrid(np.arange(640), [100, 333]), -1).reshape(-1, 2)
    pix = np.concatenate([pix, rows])
    st = P.compare_render(out, rr.render(P.ROOM_CAM, T, pixels=pix), pixels=pix,
                          name="room volume", roots=(rr, P.ROOM_CAM, T))
    assert st["hits"] > 1000


def test_volume_end_to_end_tiny(dtsdf, tiny_blobs):
    """GPU combine + GPU render against oracle combine + oracle render."""
    blob = tiny_blobs[1]
    gm = dtsdf.Map(P.tiny_gpu_params(dtsdf))
    gm.load(blob)
    src = O.OracleMap(P.tiny_oracle_params())
    src.load(blob)
    T = synth.tiny_render_pose(1.0)
    vol = dtsdf.Volume(gm, brick_capacity=1024, hash_buckets=1 << 12)
    vol.combine(gm, P.TINY_CAM, T)
    ref = _oracle_volume(P.tiny_oracle_params)
    ref.combine(src, P.TINY_CAM, T)
    out = P.to_numpy_out(vol.render(P.TINY_CAM, T, z_far=2.5))
    o = ref.render(P.TINY_CAM, T, z_far=2.5, classify=False)
    gmask = out["mask"].ravel() > 0
    both = gmask & (o.mask > 0)
    dz = np.abs(out["depth"].ravel()[both] - o.depth[both])
    mism = float((gmask != (o.mask > 0)).mean())
    print(f"[volume end-to-end] hits {int(both.sum())} mask mismatch {mism:.5f} "
          f"depth median {np.median(dz):.2e} p99 {np.percentile(dz, 99):.2e}", flush=True)
    assert both.sum() > 3000 and mism < 2e-3
    assert np.median(dz) < 1e-6 and np.percentile(dz, 99) < P.DEPTH_TOL


def test_volume_render_batch_matches_single(dtsdf, tiny_blobs):
    gm = dtsdf.Map(P.tiny_gpu_params(dtsdf))
    src = O.OracleMap(P.tiny_oracle_params())
    src.load(tiny_blobs[1])
    T = synth.tiny_render_pose(0.3)
    ref = _oracle_volume(P.tiny_oracle_params)
    ref.combine(src, P.TINY_CAM, T)
    vol = dtsdf.Volume(gm, brick_capacity=1024, hash_buckets=1 << 12)
    vol.load(ref.export())
    views = []
    singles = []
    for k, phi in enumerate((0.3, 0.35, 0.25)):
        Tk = synth.tiny_render_pose(phi)
        cam = P.TINY_CAM if k != 1 else P.TINY_CAM.level(1)
        singles.append(vol.render(cam, Tk, z_far=2.5))
        out = {key: torch.empty_like(v) for key, v in singles[-1].items()}
        views.append((cam, Tk, 0.2, 2.5, out))
    vol.render_batch(views)
    torch.cuda.synchronize()
    for s, (_, _, _, _, out) in zip(singles, views):
        for key in s:
            assert torch.equal(s[key], out[key]), key


def test_volume_argument_checks(dtsdf, tiny_blobs):
    gm = dtsdf.Map(P.tiny_gpu_params(dtsdf))
    gm.load(tiny_blobs[0])
    vol = dtsdf.Volume(gm, brick_capacity=1024, hash_buckets=1 << 12)
    T = synth.tiny_render_pose(0.3)
    with pytest.raises(dtsdf.DtsdfError):
        vol.combine(vol, P.TINY_CAM, T)                  # a volume is not a source
    with pytest.raises(dtsdf.DtsdfError):
        vol.combine(gm, P.TINY_CAM, T, margin=-1.0)
    with pytest.raises(TypeError):
        vol.integrate(None, None, P.TINY_CAM, T)
    bad = dict(tiny_blobs[0])
    with pytest.raises(dtsdf.DtsdfError):
        vol.load(bad)                                    # six-direction keys
    small = dtsdf.Volume(gm, brick_capacity=8, hash_buckets=1 << 12)
    with pytest.raises(dtsdf.DtsdfError) as e:
        small.combine(gm, P.TINY_CAM, T)
    assert e.value.status == dtsdf.E_CAPACITY
