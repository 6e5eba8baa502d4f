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
# cell face can take normal and colour from the neighbouring cell, and where the combination
# weights are near zero normal and colour can change within eps_root beyond the root.
MASK_FLAGS = O.NEAR_ZERO | O.NEAR_FACE | O.BRANCH
DEPTH_FLAGS = MASK_FLAGS | O.AMBIGUOUS
ROOT_FLAGS = O.ROOT_FACE | O.ROOT_BRANCH | O.ROOT_SHADE
SHADE_FLAGS = DEPTH_FLAGS | ROOT_FLAGS
# Upper bound on the share of compared pixels whose hit decision is exempt (the exception is
# meant for rays that graze a zero crossing, not for a sizeable part of the image), and on the
# share exempt from the depth comparison because their lattice bracket holds several roots
# (any of them is a valid result; verify_roots checks that the GPU found one)
MAX_FLAGGED_SHARE = 0.01
MAX_AMBIGUOUS_SHARE = 0.05
# ... and on the share exempt from the normal and colour comparison because the outputs at
# the root are not fixed at the refinement's resolution (ROOT_FLAGS)
# (the room's box edges and 5 mm plates put about 2 % of the roots where every combination
# weight is near zero)
MAX_ROOT_SHARE = 0.03
# ... and on the share whose bracket the oracle sampled as holding one root while the GPU
# converged to another, confirmed, root of it
MAX_FOUND_SHARE = 1e-3


def compare_render(gpu: dict, ref, pixels=None, *, W=None, name="", roots=None):
    """Compares GPU render outputs (dict of CPU numpy arrays, full images) with oracle
    outputs for `pixels` ((n,2) u,v; None: all).  Returns a stats dict; raises on failure.

    The hit mask must be equal except where a lattice sample up to the hit is flagged
    (MASK_FLAGS); depth is compared where both hit outside DEPTH_FLAGS, normal and colour
    outside SHADE_FLAGS.  At most MAX_FLAGGED_SHARE of the pixels may be exempt from the mask
    comparison and at most MAX_AMBIGUOUS_SHARE may have an ambiguous bracket.

    roots = (oracle map, camera, pose): the GPU's depth at every AMBIGUOUS pixel must be a
    root of the bracket (verify_roots); and a depth further than ROOT_WINDOW from the oracle's
    where the oracle found one root is accepted as another root of the bracket (which then
    holds several, more than the oracle's sampling of it showed) if verify_roots confirms it,
    at most MAX_FOUND_SHARE of the pixels; such pixels are then exempt like AMBIGUOUS ones."""
    if pixels is None:
        H, Wd = gpu["mask"].shape
        vv, uu = np.mgrid[0:H, 0:Wd]
        pixels = np.stack([uu.ravel(), vv.ravel()], 1)
    u, v = pixels[:, 0], pixels[:, 1]
    gm = gpu["mask"][v, u].astype(bool)
    om = ref.mask.astype(bool)
    fl = ref.flags.astype(int)
    found = not_root = None
    if roots is not None:
        om_, cam_, T_ = roots
        both0 = gm & om & ((fl & MASK_FLAGS) == 0)
        dz0 = np.abs(gpu["depth"][v, u].astype(np.float64) - ref.depth)
        # depths further apart than the refinement's resolution: another root, if confirmed
        # (else judged by the depth tolerance below)
        miss = np.where(both0 & ((fl & O.AMBIGUOUS) == 0) & (dz0 > ROOT_WINDOW))[0]
        good = verify_roots(gpu, ref, pixels, miss, om_, cam_, T_)
        fl[miss[good]] |= O.AMBIGUOUS
        found = int(good.sum())
        amb = np.where(both0 & ((ref.flags & O.AMBIGUOUS) != 0))[0]
        not_root = int((~verify_roots(gpu, ref, pixels, amb, om_, cam_, T_)).sum())
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
        bad_n = np.where(shade)[0][ang > NORMAL_TOL_DEG]
        bad_n = bad_n[np.argsort(-ang[ang > NORMAL_TOL_DEG])]   # worst first
    if "vertex" in gpu:
        gv = np.stack([gpu["vertex"][k][v, u] for k in range(3)], 1)[both]
        st["vertex_max"] = float(np.abs(gv - ref.vertex[both]).max()) if gv.size else 0.0
    if "rgba" in gpu:
        gc = gpu["rgba"][v, u][shade].astype(int)
        oc = ref.rgba[shade].astype(int)
        st["alpha_mismatch"] = int((gc[:, 3] != oc[:, 3]).sum())
        bad_a = np.where(shade)[0][gc[:, 3] != oc[:, 3]]
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
    st["ambiguous"] = int(((ref.flags & O.AMBIGUOUS) != 0).sum())
    st["root_exempt"] = int(((fl & ROOT_FLAGS) != 0).sum())
    if roots is not None:
        st["ambiguous_found"] = found
        st["ambiguous_not_root"] = not_root
        if not_root:
            problems.append("ambiguous not at a root")
        if found > MAX_FOUND_SHARE * st["n"]:
            problems.append("found ambiguous share")
    if st["flagged_mask"] > MAX_FLAGGED_SHARE * st["n"]:
        problems.append("flagged share")
    if st["ambiguous"] > MAX_AMBIGUOUS_SHARE * st["n"]:
        problems.append("ambiguous share")
    if st["root_exempt"] > MAX_ROOT_SHARE * st["n"]:
        problems.append("root exemption share")
    print(f"[render parity {name}] {st}", flush=True)
    if problems:
        # the first offending pixels, with both sides' values and the oracle's flags
        for lab, idx in (("normal", locals().get("bad_n")), ("alpha", locals().get("bad_a")),
                         ("mask", np.where(mism)[0]),
                         ("depth", np.where(both)[0][dz > DEPTH_TOL])):
            if idx is None or not len(idx):
                continue
            for i in idx[:6]:
                g = {k: (gpu[k][:, v[i], u[i]] if gpu[k].ndim == 3 and k != "rgba"
                         else gpu[k][v[i], u[i]]) for k in ("depth", "normal", "rgba")
                     if k in gpu}
                print(f"  {lab} pixel ({u[i]}, {v[i]}): gpu {g} | oracle depth "
                      f"{ref.depth[i]!r} normal {ref.normal[i]} rgba "
                      f"{getattr(ref, 'rgba', None)[i] if hasattr(ref, 'rgba') else None} "
                      f"flags {int(fl[i])} khit {int(ref.khit[i])}", flush=True)
    assert not problems, f"{name}: {problems} {st}"
    return st


ROOT_WINDOW = 2e-6   # metres along the ray: refinement tolerance plus float32 depth rounding


def verify_roots(gpu: dict, ref, pixels, sel, om, cam, T, *, z_near=0.2):
    """Whether the GPU's depth at pixels[sel] is a root of the oracle's f inside the oracle's
    lattice bracket: the GPU's ray parameter lies in [t_{k-1}, t_k] of the oracle's hit
    index k, and within ROOT_WINDOW of it f changes from positive (or undefined, counted as
    free space) to non-positive between two samples of the window (81 even ones plus both
    sides of every cell face it crosses, where f may jump).  Returns a bool array."""
    if sel.size == 0:
        return np.zeros(0, bool)
    u, v = pixels[sel, 0], pixels[sel, 1]
    step = 0.5 * om.params.voxel if om.params.step is None else om.params.step
    dc = np.stack([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy, np.ones(sel.size)], 1)
    rc = dc / np.linalg.norm(dc, axis=1, keepdims=True)
    rw = rc @ T[:3, :3].T
    o = T[:3, 3]
    tg = gpu["depth"][v, u].astype(np.float64) / rc[:, 2]
    t0 = z_near / rc[:, 2]
    ta = t0 + (ref.khit[sel] - 1) * step
    tb = t0 + ref.khit[sel] * step
    inside = (tg >= ta - ROOT_WINDOW) & (tg <= tb + ROOT_WINDOW)
    ok = np.zeros(sel.size, bool)
    vox = om.params.voxel
    for i in range(sel.size):
        ts = list(tg[i] + np.linspace(-ROOT_WINDOW, ROOT_WINDOW, 81))
        for k in range(3):
            if rw[i, k] == 0.0:
                continue
            xa = (o[k] + (tg[i] - ROOT_WINDOW) * rw[i, k]) / vox
            xb = (o[k] + (tg[i] + ROOT_WINDOW) * rw[i, k]) / vox
            for fc in range(int(math.ceil(min(xa, xb))), int(math.floor(max(xa, xb))) + 1):
                tf = (fc * vox - o[k]) / rw[i, k]
                ts += [tf - 1e-9, tf + 1e-9]
        ts = np.sort(np.array(ts))
        f, d, _ = om.eval(o[None] + ts[:, None] * rw[i][None], rw[i])
        pos = ~d | (f > 0)
        neg = d & (f <= 0)
        ok[i] = bool(np.any(pos[:-1] & neg[1:]))
    return inside & ok


def check_ambiguous_roots(gpu: dict, ref, pixels, om, cam, T, *, name=""):
    """For pixels whose bracket holds several roots (AMBIGUOUS, both sides hit): the GPU's
    depth is one of them (verify_roots).  Returns the count."""
    u, v = pixels[:, 0], pixels[:, 1]
    sel = np.where(((ref.flags & O.AMBIGUOUS) != 0) & (ref.mask > 0) &
                   (gpu["mask"][v, u] > 0) & ((ref.flags & MASK_FLAGS) == 0))[0]
    good = verify_roots(gpu, ref, pixels, sel, om, cam, T)
    bad = ~good
    print(f"[ambiguous roots {name}] {sel.size} pixels, {int(bad.sum())} not at a root", flush=True)
    assert not bad.any(), (name, pixels[sel][bad][:5])
    return int(sel.size)


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


def twist_between(Ta, Tb, dim):
    """Twist xi (translation part, rotation vector, and for dim 7 log scale) with
    exp(xi) Tb = Ta, in the parametrisation of the ICP step (left update)."""
    import scipy.linalg
    G = np.real(scipy.linalg.logm(np.asarray(Ta, np.float64) @ np.linalg.inv(Tb)))
    A = G[:3, :3]
    sigma = np.trace(A) / 3.0
    W = A - sigma * np.eye(3)
    xi = [G[0, 3], G[1, 3], G[2, 3], W[2, 1], W[0, 2], W[1, 0]]
    return np.array(xi + ([sigma] if dim == 7 else []))


# change of the RMS point-to-plane residual that a pose difference along the weak directions
# of an ill-conditioned registration may cause: the translation bar of the pose (1e-5 m), a
# fiftieth of the live frames' depth noise (0.5 mm), below which two poses fit the frame
# indistinguishably
RESID_TOL = 1e-5


def pose_parity(live, cam, gpu_levels, oracle_levels, T_g, dT0, dim, *, name=""):
    """Pose parity of a registration on a poorly conditioned scene (the tiny sphere-and-plate
    scene leaves rotation about the sphere centre almost free: cond(H) 1e4 .. 4e4).

    (1) The oracle's ICP on the GPU's own model pyramid `gpu_levels` (the reduction and
        solve alone): the pose difference within 1e-5 in the well-conditioned eigen-directions
        of the finest level's H (eigenvalues above 1/100 of the largest), and the change of
        the RMS residual it causes within RESID_TOL; the part along the weak directions
        (float32 sums amplified by cond(H)) is reported.
    (2) The oracle's ICP on its own renders `oracle_levels` (render and registration
        together) may stop at another point of the weak valley: the GPU's pose fits the live
        frame no worse than the oracle's (RMS residual at most 0.1 mm above it).
    Returns the stats; failures are listed under "fails"."""
    T_s, _ = O.icp(live, cam, gpu_levels, dT0, dim=dim)
    ds = twist_between(T_g, T_s, dim)
    LV, LN, LOK = O.vertex_normal_map(live, cam)
    H, _, _, cnt = O.associate_reduce(LV, LN, LOK, *gpu_levels[0][:3], cam, T_s, dim)
    ev, evec = np.linalg.eigh(H)
    strong = ev >= ev[-1] / 100.0
    cs = evec.T @ ds
    T_o, _ = O.icp(live, cam, oracle_levels, dT0, dim=dim)
    de = twist_between(T_g, T_o, dim)
    _, _, err_o, cnt_o = O.associate_reduce(LV, LN, LOK, *oracle_levels[0][:3], cam, T_o, dim)
    _, _, err_g, cnt_g = O.associate_reduce(LV, LN, LOK, *oracle_levels[0][:3], cam, T_g, dim)
    st = dict(cond=float(ev[-1] / ev[0]), weak=int((~strong).sum()),
              same_strong=float(np.linalg.norm(cs[strong])),
              same_weak=float(np.linalg.norm(cs[~strong])),
              same_resid=math.sqrt(max(float(ds @ H @ ds), 0.0) / cnt),
              own_rot=float(np.linalg.norm(de[3:6])), own_trans=float(np.linalg.norm(de[:3])),
              rms_g=math.sqrt(err_g / cnt_g), rms_o=math.sqrt(err_o / cnt_o), fails=[])
    if dim == 7:
        st["own_log_scale"] = float(abs(de[6]))
    if not (st["same_strong"] < 1e-5 and st["same_resid"] < RESID_TOL):
        st["fails"].append(("same maps", st["same_strong"], st["same_resid"]))
    if not st["rms_g"] < st["rms_o"] + 1e-4:
        st["fails"].append(("own renders: GPU pose fits worse", st["rms_g"], st["rms_o"]))
    print(f"[pose parity {name}] cond(H) {st['cond']:.3g} ({st['weak']} weak of {dim}); same "
          f"maps: well-conditioned part {st['same_strong']:.2e}, weak part "
          f"{st['same_weak']:.2e}, residual change {st['same_resid']:.2e} m | own renders: "
          f"rot {st['own_rot']:.2e} rad trans {st['own_trans']:.2e} m, rms residual "
          f"{st['rms_g'] * 1e3:.4f} mm (GPU pose) vs {st['rms_o'] * 1e3:.4f} mm (oracle pose)",
          flush=True)
    return st


def rotation_angle(R):
    return math.acos(max(-1.0, min(1.0, (np.trace(R) - 1.0) / 2.0)))
