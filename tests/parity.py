"""Shared helpers of the GPU parity tests: workloads, map parameters and comparators.

Tolerances (from the targets of the method's hot path): hit mask equal outside the grazing
set G flagged by the oracle, depth within 1e-4 m, normals within 0.5 degrees, colour within
one 8-bit step per channel, pose within 1e-5 rad and 1e-5 m.
"""
import math

import numpy as np

import synth
from oracle import oracle as O

DEPTH_TOL = 1e-4
NORMAL_TOL_DEG = 0.5
COLOR_TOL = 1

TINY_CAM = synth.scenes.TINY_CAMERA
ROOM_CAM = synth.scenes.ROOM_CAMERA


def tiny_oracle_params(**kw):
    return O.MapParams(voxel=0.01, tau=0.04, dense_lo=synth.scenes.TINY_DENSE_LO,
                       dense_hi=synth.scenes.TINY_DENSE_HI, **kw)


def tiny_gpu_params(dtsdf, **kw):
    return dtsdf.Params(voxel_size=0.01, truncation=0.04, brick_capacity=4096,
                        hash_buckets=1 << 12, dense_lo=synth.scenes.TINY_DENSE_LO,
                        dense_hi=synth.scenes.TINY_DENSE_HI, **kw)


def room_oracle_params(**kw):
    return O.MapParams(voxel=0.005, tau=0.02, **kw)


def room_gpu_params(dtsdf, capacity=1 << 19, buckets=1 << 20, **kw):
    return dtsdf.Params(voxel_size=0.005, truncation=0.02, brick_capacity=capacity,
                        hash_buckets=buckets, **kw)


# Flags that exempt a pixel from a comparison.  The hit decision depends only on the lattice
# samples up to the hit (near-zero value, cell-face, thresholded weight factor); an
# ambiguous bracket can move the root (depth, normal, colour); a root within eps_root of a
# cell face can take normal and colour from the neighbouring cell.
MASK_FLAGS = O.NEAR_ZERO | O.NEAR_FACE | O.BRANCH
DEPTH_FLAGS = MASK_FLAGS | O.AMBIGUOUS
SHADE_FLAGS = DEPTH_FLAGS | O.ROOT_FACE
# Upper bound on the share of compared pixels that any flag exempts (the exception is meant
# for rays that graze a zero crossing, not for a sizeable part of the image)
MAX_FLAGGED_SHARE = 0.01


def compare_render(gpu: dict, ref, pixels=None, *, W=None, name=""):
    """Compares GPU render outputs (dict of CPU numpy arrays, full images) with oracle
    outputs for `pixels` ((n,2) u,v; None: all).  Returns a stats dict; raises on failure.

    The hit mask must be equal except where a lattice sample up to the hit is flagged
    (MASK_FLAGS); depth is compared where both hit outside DEPTH_FLAGS, normal and colour
    outside SHADE_FLAGS.  At most MAX_FLAGGED_SHARE of the pixels may carry any flag."""
    if pixels is None:
        H, Wd = gpu["mask"].shape
        vv, uu = np.mgrid[0:H, 0:Wd]
        pixels = np.stack([uu.ravel(), vv.ravel()], 1)
    u, v = pixels[:, 0], pixels[:, 1]
    gm = gpu["mask"][v, u].astype(bool)
    om = ref.mask.astype(bool)
    fl = ref.flags.astype(int)
    g_mask = (fl & MASK_FLAGS) != 0
    g_depth = (fl & DEPTH_FLAGS) != 0
    g_shade = (fl & SHADE_FLAGS) != 0
    st = dict(n=len(u), hits=int(om.sum()), flagged=int((fl != 0).sum()),
              flagged_mask=int(g_mask.sum()), flagged_share=float((fl != 0).mean()) if len(u) else 0.0)
    mism = (gm != om) & ~g_mask
    st["mask_mismatch"] = int(mism.sum())
    st["mask_mismatch_incl_flagged"] = int((gm != om).sum())
    both = gm & om & ~g_depth
    st["compared"] = int(both.sum())
    dz = np.abs(gpu["depth"][v, u][both] - ref.depth[both])
    st["depth_max"] = float(dz.max()) if dz.size else 0.0
    shade = gm & om & ~g_shade
    if "normal" in gpu:
        gn = np.stack([gpu["normal"][k][v, u] for k in range(3)], 1)[shade]
        on = ref.normal[shade]
        cosang = np.clip((gn * on).sum(1) / np.maximum(np.linalg.norm(gn, axis=1), 1e-30), -1, 1)
        ang = np.degrees(np.arccos(cosang))
        st["normal_max_deg"] = float(ang.max()) if ang.size else 0.0
    if "vertex" in gpu:
        gv = np.stack([gpu["vertex"][k][v, u] for k in range(3)], 1)[both]
        st["vertex_max"] = float(np.abs(gv - ref.vertex[both]).max()) if gv.size else 0.0
    if "rgba" in gpu:
        gc = gpu["rgba"][v, u][shade].astype(int)
        oc = ref.rgba[shade].astype(int)
        st["alpha_mismatch"] = int((gc[:, 3] != oc[:, 3]).sum())
        cb = (gc[:, 3] == 255) & (oc[:, 3] == 255)
        st["color_max"] = int(np.abs(gc[cb, :3] - oc[cb, :3]).max()) if cb.any() else 0
    problems = []
    if st["mask_mismatch"]:
        problems.append("mask")
    if st["depth_max"] > DEPTH_TOL:
        problems.append("depth")
    if st.get("vertex_max", 0) > DEPTH_TOL:
        problems.append("vertex")
    if st.get("normal_max_deg", 0) > NORMAL_TOL_DEG:
        problems.append("normal")
    if st.get("color_max", 0) > COLOR_TOL or st.get("alpha_mismatch", 0):
        problems.append("color")
    if st["flagged"] > MAX_FLAGGED_SHARE * st["n"]:
        problems.append("flagged share")
    print(f"[render parity {name}] {st}", flush=True)
    assert not problems, f"{name}: {problems} {st}"
    return st


def to_numpy_out(out: dict) -> dict:
    return {k: v.cpu().numpy() for k, v in out.items()}


def compare_maps(gpu_blob: dict, orc_blob: dict, *, n_frames: int, name=""):
    """Voxel-wise comparison of two exported maps on their common bricks; voxels the oracle
    flags as borderline are skipped.

    Weights: the float32 path carries ~5e-7 absolute error per fused weight (float32
    normals feeding w_dir and w_angle) plus float32 rounding of the running sum, so weights
    are compared with |dw| <= 1e-6 * n_frames + 2e-5 * w.  Distances: voxels whose total
    weight is below 1e-2 average few tiny, relatively uncertain weights and are compared
    at 1e-3; the others at 5e-5.  Colours: one 8-bit step (a tie on the rounding of the
    running colour average may fall either way)."""
    gk = {tuple(k): i for i, k in enumerate(gpu_blob["keys"])}
    ok = {tuple(k): i for i, k in enumerate(orc_blob["keys"])}
    common = sorted(set(gk) & set(ok))
    gi = np.array([gk[c] for c in common], np.int64)
    oi = np.array([ok[c] for c in common], np.int64)
    border = orc_blob["border"][oi].astype(bool)
    keep = ~border
    gw, ow = gpu_blob["w"][gi][keep], orc_blob["w"][oi][keep]
    wtol = 1e-6 * n_frames + 2e-5 * np.maximum(gw, ow)
    ds = np.abs(gpu_blob["sdf"][gi] - orc_blob["sdf"][oi])[keep]
    heavy = ow >= 1e-2
    st = dict(common=len(common), only_gpu=len(set(gk) - set(ok)),
              only_oracle=len(set(ok) - set(gk)), border=int(border.sum()),
              sdf_max_heavy=float(ds[heavy].max()) if heavy.any() else 0.0,
              sdf_max_light=float(ds[~heavy].max()) if (~heavy).any() else 0.0,
              w_excess=float((np.abs(gw - ow) / wtol).max()) if gw.size else 0.0,
              w_zero_mismatch=int(((gw > 0) != (ow > 0)).sum()))
    ok_ = st["sdf_max_heavy"] < 5e-5 and st["sdf_max_light"] < 1e-3 and st["w_excess"] <= 1.0 \
        and st["w_zero_mismatch"] == 0
    if "rgb" in gpu_blob and "rgb" in orc_blob:
        gc = gpu_blob["rgb"][gi][keep].astype(int)
        oc = orc_blob["rgb"][oi][keep].astype(int)
        st["rgb_max"] = int(np.abs(gc - oc).max()) if gc.size else 0
        gwc, owc = gpu_blob["wc"][gi][keep], orc_blob["wc"][oi][keep]
        ctol = 1e-6 * n_frames + 2e-5 * np.maximum(gwc, owc)
        st["wc_excess"] = float((np.abs(gwc - owc) / ctol).max()) if gwc.size else 0.0
        ok_ = ok_ and st["rgb_max"] <= COLOR_TOL and st["wc_excess"] <= 1.0
    st["ok"] = bool(ok_)
    print(f"[map parity {name}] {st}", flush=True)
    return st


def random_pixels(cam, n, seed):
    rng = np.random.default_rng(seed)
    u = rng.integers(0, cam.width, n)
    v = rng.integers(0, cam.height, n)
    return np.stack([u, v], 1)


def rotation_angle(R):
    return math.acos(max(-1.0, min(1.0, (np.trace(R) - 1.0) / 2.0)))
