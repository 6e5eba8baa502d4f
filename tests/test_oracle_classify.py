"""The oracle's exemption flags for shading (CPU only).

A renderer that refines the root to a tolerance of 1e-6 m ends its bracket inside the
surface, up to that far beyond the root, and takes normal and colour there.  Outside the
pixels the oracle exempts from the normal and colour comparison (SHADE_FLAGS), the shading
at such an end point must agree with the oracle's output to the comparison tolerances; and
the exemption must be needed somewhere (it is not empty where the combination weights are
near zero), so that it marks exactly what it claims."""
import numpy as np

import synth
from oracle import oracle as O
from tests import parity as P


def _view():
    om = O.OracleMap(P.tiny_oracle_params())
    for f in synth.tiny_frames(10):
        om.integrate(f["depth"], f["rgb"], P.TINY_CAM, f["T_wc"])
    sensors = synth.serving_sensors()
    w = [x for x in synth.serving_workload(40, seed=25) if x["sensor"] == 2][0]
    cam, _ = sensors[2]
    return om, cam, w["T_model"]


def test_shading_within_refinement_tolerance():
    om, cam, T = _view()
    vv, uu = np.mgrid[0:cam.height:2, 0:cam.width]   # every second row of the 848x480 view
    pix = np.stack([uu.ravel(), vv.ravel()], 1)
    ref = om.render(cam, T, pixels=pix)
    hit = np.where(ref.mask > 0)[0]
    u, v = pix[hit, 0], pix[hit, 1]
    dc = np.stack([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy, np.ones(hit.size)], 1)
    rc = dc / np.linalg.norm(dc, axis=1, keepdims=True)
    rw = rc @ T[:3, :3].T
    exempt = (ref.flags[hit] & P.SHADE_FLAGS) != 0
    ref_nw = ref.normal[hit] @ T[:3, :3].T          # camera -> world
    needed = 0
    for delta in (2.5e-7, 5e-7, 1e-6):
        x = T[:3, 3][None] + (ref.thit[hit] + delta)[:, None] * rw
        n, rgb, has_n, has_c = om.shade(x, rw)
        ang = np.degrees(np.arccos(np.clip((n * ref_nw).sum(1), -1, 1)))
        ref_c = ref.rgba[hit, 3] == 255
        dcol = np.abs(np.clip(np.rint(rgb), 0, 255) - ref.rgba[hit, :3]).max(1)
        bad = ~has_n | (ang > P.NORMAL_TOL_DEG) | (has_c != ref_c) | \
            (has_c & ref_c & (dcol > P.COLOR_TOL))
        assert not (bad & ~exempt).any(), (delta, pix[hit][bad & ~exempt][:5],
                                          ang[bad & ~exempt][:5])
        needed += int((bad & exempt).sum())
    print(f"{hit.size} hits, {int(exempt.sum())} exempt from shading, {needed} of them "
          f"would fail within the tolerance")
    assert needed > 0
    # the exemption is meant for a small part of the image
    assert exempt.mean() < 0.02


def test_root_verification():
    """verify_roots, the check that a renderer's depth is a root of the oracle's bracket where
    several are valid: the oracle's own roots pass; a depth moved off the root fails; and in a
    bracket with several roots another root (found here by a fine scan) passes."""
    om, cam, T = _view()
    vv, uu = np.mgrid[0:cam.height:4, 0:cam.width]
    pix = np.stack([uu.ravel(), vv.ravel()], 1)
    ref = om.render(cam, T, pixels=pix)
    gpu = dict(depth=np.zeros((cam.height, cam.width), np.float32),
               mask=np.zeros((cam.height, cam.width), np.uint8))
    u, v = pix[:, 0], pix[:, 1]
    gpu["depth"][v, u] = ref.depth
    gpu["mask"][v, u] = ref.mask
    st = P.compare_render(gpu, ref, pixels=pix, name="oracle itself", roots=(om, cam, T))
    assert st["ambiguous"] > 0 and st["ambiguous_not_root"] == 0 and st["ambiguous_found"] == 0
    amb = np.where(((ref.flags & O.AMBIGUOUS) != 0) & ((ref.flags & P.MASK_FLAGS) == 0) &
                   (ref.mask > 0))[0]
    step = 0.5 * om.params.voxel
    moved = other = 0
    for i in amb:
        dc = np.array([(u[i] - cam.cx) / cam.fx, (v[i] - cam.cy) / cam.fy, 1.0])
        rc = dc / np.linalg.norm(dc)
        rw = T[:3, :3] @ rc
        t0 = 0.2 / rc[2]
        ts = t0 + (ref.khit[i] - 1) * step + np.linspace(0, step, 20001)
        f, d, _ = om.eval(T[:3, 3][None] + ts[:, None] * rw[None], rw)
        pos = ~d | (f > 0)
        ch = np.where(pos[:-1] & d[1:] & (f[1:] <= 0))[0]
        far = ch[np.abs(ts[ch] - ref.thit[i]) > 1e-4]
        if far.size and other < 5:
            # another root of the same bracket: accepted
            g = {k: a.copy() for k, a in gpu.items()}
            g["depth"][v[i], u[i]] = 0.5 * (ts[far[0]] + ts[far[0] + 1]) * rc[2]
            good = P.verify_roots(g, ref, pix, np.array([i]), om, cam, T)
            assert good.all(), (u[i], v[i])
            other += 1
        if moved < 5:
            # a depth off every root: rejected
            roots_t = 0.5 * (ts[ch] + ts[ch + 1])
            cand = ts[np.argmax(np.min(np.abs(ts[:, None] - roots_t[None]), 1))]
            g = {k: a.copy() for k, a in gpu.items()}
            g["depth"][v[i], u[i]] = cand * rc[2]
            assert not P.verify_roots(g, ref, pix, np.array([i]), om, cam, T).any()
            moved += 1
    assert other > 0 and moved > 0
