"""Parity of input preprocessing (Sec. 7, Sec. 8 parameters) and the post-fusion error with the
FP64 oracle, through the C ABI.

Depth filter: the kept-pixel mask is compared exactly (the support tests are exact on both
sides), values within 2e-6 m (float32 weights and sums, accumulated relative to the centre
depth: a weighted mean of offsets below ~0.1 m carries ~1e-6 m, plus the output rounding).
Normal filter: the valid mask exactly, components within 2e-5 (float32 weights over up to 289
taps).  Post-fusion error: the count exactly, the mean to 1e-12 relative (float64 sums)."""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import parity as P

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dtsdf():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2301_12796_amd import dtsdf as lib
    return lib


def _noisy_depth(W=640, H=480, seed=4, outliers=0.005, holes=0.01):
    """Room frame with quadratic noise, then seeded outliers (uniform 0.3-5 m) and holes."""
    cam = P.ROOM_CAM
    d = synth.render_frame(synth.room_scene(), cam, synth.room_pose(60), noise="quadratic",
                           sigma=0.0012, seed=seed)["depth"][:H, :W].copy()
    rng = np.random.default_rng(seed)
    m = rng.random(d.shape)
    d[m < outliers] = rng.uniform(0.3, 5.0, int((m < outliers).sum())).astype(np.float32)
    d[(m >= outliers) & (m < outliers + holes)] = 0.0
    return np.ascontiguousarray(d, np.float32)


def _f32(x):
    return float(np.float32(x))


@pytest.mark.parametrize("shape,params", [
    ((640, 480), dict()),                                      # Sec. 8 values
    ((203, 157), dict(radius=8, min_support=3, sigma_d=3.0)),  # ragged tiles, largest window
    ((203, 157), dict(radius=0)),                              # support filter only
    ((203, 157), dict(min_support=0)),                         # bilateral only
])
def test_depth_filter_matches_oracle(dtsdf, shape, params):
    W, H = shape
    d = _noisy_depth(W, H)
    p = dtsdf.DepthFilterParams(**params)
    out = dtsdf.depth_filter(torch.from_numpy(d).cuda(), p).cpu().numpy()
    ref = O.depth_support_filter(d, _f32(p.support_rel), p.min_support) \
        if p.min_support > 0 else d.astype(np.float64)
    if p.radius > 0:
        ref = O.bilateral_depth(ref, _f32(p.sigma_d), _f32(p.sigma_r), p.radius)
    kept = out > 0
    err = np.abs(out - ref)[kept]
    print(f"[depth filter {shape} {params}] kept {kept.mean():.4f} of pixels, removed "
          f"{int(((d > 0) & ~kept).sum())}, max err {err.max():.2e} m", flush=True)
    assert np.array_equal(kept, ref > 0)
    assert err.max() < 2e-6
    if p.min_support > 0:
        assert ((d > 0) & ~kept).sum() > 0.5 * 0.005 * W * H     # outliers were removed


def test_depth_filter_empty_and_invalid(dtsdf):
    z = torch.zeros((48, 64), dtype=torch.float32, device="cuda")
    assert not dtsdf.depth_filter(z).any()
    with pytest.raises(dtsdf.DtsdfError):
        dtsdf.depth_filter(z, dtsdf.DepthFilterParams(radius=9))
    with pytest.raises(dtsdf.DtsdfError):
        dtsdf.depth_filter(z, dtsdf.DepthFilterParams(sigma_r=0.0))


@pytest.mark.parametrize("radius,sigma_r", [(5, 5.0), (8, 20.0)])
def test_normal_filter_matches_oracle(dtsdf, radius, sigma_r):
    cam = P.ROOM_CAM
    d = dtsdf.depth_filter(torch.from_numpy(_noisy_depth()).cuda())
    _, n = dtsdf.vertex_normal(d, cam)
    out = dtsdf.normal_filter(n, 2.5, sigma_r, radius).cpu().numpy().transpose(1, 2, 0)
    N = n.cpu().numpy().transpose(1, 2, 0).astype(np.float64)
    ref = O.bilateral_normal(N, 2.5, sigma_r, radius)
    valid = np.any(out != 0, axis=-1)
    err = np.abs(out - ref).max(axis=-1)[valid]
    print(f"[normal filter r={radius} sr={sigma_r}] valid {valid.mean():.4f}, max err "
          f"{err.max():.2e}", flush=True)
    assert np.array_equal(valid, np.any(ref != 0, axis=-1))
    assert err.max() < 2e-5
    np.testing.assert_allclose(np.linalg.norm(out[valid], axis=-1), 1.0, atol=1e-6)


@pytest.mark.parametrize("shape,offset", [((640, 480), 0), ((203, 157), 0), ((203, 157), 1)])
def test_depth_error_matches_oracle(dtsdf, shape, offset):
    """Aligned images take the float4 path (with a ragged tail when W*H is not a multiple
    of four); an image starting one float in takes the scalar path."""
    W, H = shape
    a = _noisy_depth(W, H, seed=4)
    b = _noisy_depth(W, H, seed=5)
    ta = torch.zeros(W * H + offset, dtype=torch.float32, device="cuda")
    tb = torch.zeros(W * H + offset, dtype=torch.float32, device="cuda")
    ta[offset:] = torch.from_numpy(a.ravel()).cuda()
    tb[offset:] = torch.from_numpy(b.ravel()).cuda()
    mae, n = dtsdf.depth_error(ta[offset:].view(H, W), tb[offset:].view(H, W))
    ref, nr = O.post_fusion_mae(a, b)
    print(f"[depth error {shape} +{offset}] mae {mae:.6e} over {n} pixels", flush=True)
    assert n == nr and abs(mae - ref) <= 1e-12 * ref


def test_icp_on_preprocessed_frames_matches_oracle(dtsdf):
    """Three-level ICP with the live frame preprocessed (Sec. 7) on both sides, on a frame
    with seeded outliers and holes: final poses within 1e-5 rad / 1e-5 m."""
    import math
    sc = synth.room_scene()
    cam = P.ROOM_CAM
    T = synth.room_pose(60)
    live = _noisy_depth()
    dT0 = synth.perturb_pose(0.02, math.radians(2.0), np.random.default_rng(13))
    levels_o, levels_g = [], []
    for l in range(3):
        c = cam.level(l)
        f = synth.render_frame(sc, c, T)
        V = (c.pixel_rays() * f["true_depth"][..., None]).astype(np.float32)
        N = f["normal"].astype(np.float32)
        M = f["hit"].astype(np.uint8)
        levels_o.append((V.astype(np.float64), N.astype(np.float64), M, c))
        levels_g.append((torch.from_numpy(np.ascontiguousarray(V.transpose(2, 0, 1))).cuda(),
                         torch.from_numpy(np.ascontiguousarray(N.transpose(2, 0, 1))).cuda(),
                         torch.from_numpy(M).cuda(), c))
    T_o, _ = O.icp(live, cam, levels_o, dT0, preprocess=O.Preprocess())
    T_g, log = dtsdf.icp(torch.from_numpy(live).cuda(), cam, levels_g, dT0,
                         preprocess=dtsdf.Preprocess())
    ang = P.rotation_angle(T_g[:3, :3] @ T_o[:3, :3].T)
    dt = np.linalg.norm(T_g[:3, 3] - T_o[:3, 3])
    print(f"[icp preprocessed] rot {ang:.2e} rad trans {dt:.2e} m, {len(log)} steps, "
          f"|t| {np.linalg.norm(T_g[:3, 3]):.2e} m", flush=True)
    assert ang < 1e-5 and dt < 1e-5


def test_fusion_with_given_normals_matches_oracle(dtsdf):
    """dtsdf_integrate_normals against the oracle fed the same normals: analytic normals of
    the tiny scene tilted by seeded noise (about 1 degree), float32, on a sparse map; the
    allocation lies between the oracle's required and allowed sets and the voxels agree at
    the fusion bars."""
    cam = synth.scenes.TINY_CAMERA
    frames = synth.tiny_frames(6)
    gm = dtsdf.Map(dtsdf.Params(voxel_size=0.01, truncation=0.04, brick_capacity=1 << 15,
                                hash_buckets=1 << 15))
    om = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04))
    required, allowed = set(), set()
    rng = np.random.default_rng(21)
    for f in frames:
        N = f["normal"] + rng.normal(scale=0.02, size=f["normal"].shape)
        N /= np.linalg.norm(N, axis=-1, keepdims=True)
        N = np.where(f["hit"][..., None], N, 0.0).astype(np.float32)
        keys, border, alloc = om.requests(f["depth"], cam, f["T_wc"], normals=N)
        for k, b, a in zip(map(tuple, keys), border, alloc):
            allowed.add(k)
            if a and not b:
                required.add(k)
        st = gm.integrate(torch.from_numpy(f["depth"]).cuda(), torch.from_numpy(f["rgb"]).cuda(),
                          cam, f["T_wc"], stats=True,
                          normal=torch.from_numpy(np.ascontiguousarray(N.transpose(2, 0, 1))).cuda())
        assert st["dropped"] == 0
        om.integrate(f["depth"], f["rgb"], cam, f["T_wc"], normals=N.astype(np.float64))
    gb = gm.export()
    gset = set(map(tuple, gb["keys"]))
    print(f"case: fusion with given normals, {len(gset)} bricks, required {len(required)}, "
          f"allowed {len(allowed)}", flush=True)
    assert required <= gset and gset <= allowed
    st = P.compare_maps(gb, om.export(), n_frames=len(frames), name="given normals")
    assert st["ok"], st
    with pytest.raises(dtsdf.DtsdfError):
        dtsdf._check(dtsdf._lib.dtsdf_integrate_normals(gm.handle, None, None, None, None, None,
                                                         1.0, None, None), "x")
