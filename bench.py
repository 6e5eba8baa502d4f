"""Benchmark: Directional-TSDF render throughput at 640x480 on one MI355X.

Workload (the room configuration): a 4 x 4 x 3 m room with seeded boxes, spheres and 5 mm
plates; 300 synthetic 640x480 RGB-D frames (f = 525, depth noise 0.0012 z^2) along a seeded
smooth trajectory are fused into a sparse map of 8^3 blocks at 5 mm voxels (tau = 2 cm, 8-bit
colour per direction).  One step renders depth + normal + colour at all 300 trajectory poses;
`value` is rays per second over the timed steps (map and poses resident in device memory).

Printed as one JSON line, with the roofline of the render kernel (algorithmic bytes per
launch from the traced brick / bucket sets, divided by the launch duration measured with HIP
events on the launch stream) and the FP64 oracle timed on the host cores on a bounded sample.
Separately timed and reported beside it: the same views rendered 32 per persistent launch
(rays/s and that launch's roofline, bricks counted once per launch), integration ms/frame, the geometric post-fusion error
(render at every fused pose against its input depth), the live-frame preprocessing (depth
filter, normals, normal filter), three-level ICP ms/frame on preprocessed live frames
(point-to-plane, and combined with the photometric term against a keyframe), the
precision forms (f16 / i16 distance with u8 weights, fused from the same frames: rays/s and
depth against the plain render), the serving workload (p50/p99 latency and capacity of
the continuous-batching server against serial calls) and the view-dependent combined TSDF
(recombination time, one-volume render rate and depth against the direct render, and a
frame loop under the conditional-recombination policy) and the multi-sensor Sim(3)
refinement (five sensors with scaled depth registered by Levenberg-Marquardt ICP, their
scales anchored to the first sensor), and map upkeep (recycling of bricks without surface
on the fused map: bricks freed, time, render and post-fusion error before and after).
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DTSDF render rays/s at 640x480 (% HBM roofline); served p50/p99 render+ICP ms"
HBM_PEAK_GBS = 8000.0
# vector issue: each CU's four SIMDs have 16 lanes, so a wave64 VALU instruction occupies
# its SIMD for 4 cycles: 256 CUs x 4 SIMDs / 4 cycles x 2.4 GHz wave instructions per second
# (x 64 lanes x 2 flops per FMA x 2 for packed fp32 = the 157.3 TFLOP/s fp32 vector peak)
VALU_ISSUE_PEAK = 256 * 2.4e9
OUT_BYTES_PER_RAY = 4 + 12 + 4 + 1          # depth + normal + rgba + mask
BRICK_MARCH_BYTES = 512 * 8                 # (sdf, w) float32 per voxel
BRICK_COLOR_BYTES = 512 * 8                 # rgb code + colour weight per voxel
# per block a ray enters: its grid record (six brick indices, info word, hash slot: 32 B),
# its positive-cell words (64 B) and its direction-group bytes (64 B)
RECORD_BYTES = 32 + 64 + 64


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash(path):
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def read_profile(name, kernel_src):
    """The `key = value` lines of a committed rocprofv3 summary under profiles/, if it was
    taken on the current kernel source (else None)."""
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    kv = {}
    for line in open(p):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != source_hash(kernel_src):
        return None
    return kv


def read_float(kv, key):
    try:
        return float(kv[key]) if kv is not None else None
    except (KeyError, ValueError):
        return None


def roofline_block(achieved, traffic, valu_per_launch, valu_frac, mean_launch_s, ctr):
    """Roofline of the render kernel on two axes: HBM (algorithmic bytes per launch over the
    launch time, against 8 TB/s) and vector issue (VALU wave instructions per launch, from
    the committed counter summary of the same source, over the launch time, against
    VALU_ISSUE_PEAK).  `bound` names the axis with the larger fraction, whose figures fill
    achieved / peak / unit / frac; both are given under `hbm` and `alu`."""
    hbm = dict(achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS)
    alu = None
    if valu_frac is not None:
        alu = dict(achieved=valu_per_launch / mean_launch_s / 1e9, peak=VALU_ISSUE_PEAK / 1e9,
                   unit="G VALU wave-instructions/s", frac=valu_frac)
    bound = "alu" if alu is not None and alu["frac"] > hbm["frac"] else "hbm"
    top = alu if bound == "alu" else hbm
    return dict(bound=bound, achieved=top["achieved"], peak=top["peak"], unit=top["unit"],
                frac=top["frac"], traffic=traffic, hbm=hbm, alu=alu,
                valu_insts_per_launch=valu_per_launch,
                salu_insts_per_launch=read_float(ctr, "salu_insts_per_launch"),
                l2_hit_rate=read_float(ctr, "l2_hit_rate"),
                traffic_over_algorithmic=(traffic / (achieved * mean_launch_s * 1e9)
                                          if traffic is not None else None))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-icp", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-volume", action="store_true")
    ap.add_argument("--no-recycle", action="store_true")
    ap.add_argument("--no-prefuse", action="store_true",
                    help="skip fusing the frames a second time through the preprocessing")
    ap.add_argument("--batch", type=int, default=32,
                    help="views per launch of the batched render block (1: skip it)")
    ap.add_argument("--serve-requests", type=int, default=3600,
                    help="leading requests of the 120/s Poisson stream that are served")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2301_12796_amd import dtsdf

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()

    # ---- inputs: scene, frames, fused map (setup, not timed as render) -----------------
    cam = synth.scenes.ROOM_CAMERA
    sc = synth.room_scene()
    n = args.frames
    params = dtsdf.Params(voxel_size=0.005, truncation=0.02, brick_capacity=1 << 20,
                          hash_buckets=1 << 21)
    gm = dtsdf.Map(params)
    t_gen = 0.0
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    integ_ms = 0.0
    frames_dev = []          # kept for the precision-form maps
    fuse_counts = []         # per frame: bricks visited, voxels updated, colours updated
    for k in range(n):
        t = time.time()
        f = synth.scenes.render_frame(sc, cam, synth.room_pose(k, n), noise="quadratic",
                                      sigma=0.0012, seed=2000 + k, z_max=10.0, device="cuda")
        depth = torch.from_numpy(f["depth"]).to(dev)
        rgb = torch.from_numpy(f["rgb"]).to(dev)
        frames_dev.append((depth, rgb))
        t_gen += time.time() - t
        ev0.record(stream)
        ist = gm.integrate(depth, rgb, cam, synth.room_pose(k, n), stats=True)
        ev1.record(stream)
        ev1.synchronize()
        integ_ms += ev0.elapsed_time(ev1)
        fuse_counts.append((ist["visited_bricks"], ist["updated_voxels"], ist["color_voxels"]))
        if k % 50 == 0:
            log(f"fused frame {k}/{n}: {gm.info()['bricks']} bricks")
    info = gm.info()
    log(f"map: {info['bricks']} bricks, {info['blocks']} blocks, dropped {info['dropped']}")
    # fusion roofline: per updated voxel (sdf, w) read and written (16 B), per updated colour
    # (rgb code, colour weight) read and written (16 B), per visited brick its key (16 B),
    # per pixel the frame's depth, normal, colour and carving flag (20 B)
    fc = np.array(fuse_counts, np.float64)
    fuse_bytes = (fc[:, 1] * 16 + fc[:, 2] * 16 + fc[:, 0] * 16).mean() + \
        cam.width * cam.height * 20
    fuse_prof = read_profile("integrate_room_640x480_stats.txt",
                             os.path.join(ROOT, "paper_2301_12796_amd", "csrc", "integrate.hip"))
    fuse_k_us = read_float(fuse_prof, "fuse_k_average_us")
    fusion = dict(visited_bricks_per_frame=float(fc[:, 0].mean()),
                  updated_voxels_per_frame=float(fc[:, 1].mean()),
                  color_voxels_per_frame=float(fc[:, 2].mean()),
                  algorithmic_bytes_per_frame=float(fuse_bytes),
                  integrate_ms_per_frame=integ_ms / n,
                  achieved_gbs_whole_frame=float(fuse_bytes / (integ_ms / n * 1e-3) / 1e9),
                  fuse_k_average_us=fuse_k_us,
                  achieved_gbs_fuse_k=(float(fuse_bytes / (fuse_k_us * 1e-6) / 1e9)
                                       if fuse_k_us else None),
                  peak=HBM_PEAK_GBS, unit="GB/s")
    fusion["frac_whole_frame"] = fusion["achieved_gbs_whole_frame"] / HBM_PEAK_GBS
    fusion["frac_fuse_k"] = (fusion["achieved_gbs_fuse_k"] / HBM_PEAK_GBS
                             if fusion["achieved_gbs_fuse_k"] else None)
    log(f"fusion: {fc[:, 1].mean():.0f} voxels updated per frame ({fc[:, 0].mean():.0f} bricks "
        f"visited), {fuse_bytes / 1e6:.1f} MB algorithmic, {fusion['achieved_gbs_whole_frame']:.0f}"
        f" GB/s over the whole integrate call")

    poses = [synth.room_pose(k, n) for k in range(n)]
    H, W = cam.height, cam.width
    out = dict(depth=torch.empty((H, W), dtype=torch.float32, device=dev),
               normal=torch.empty((3, H, W), dtype=torch.float32, device=dev),
               rgba=torch.empty((H, W, 4), dtype=torch.uint8, device=dev),
               mask=torch.empty((H, W), dtype=torch.uint8, device=dev))

    # ---- algorithmic bytes per launch from traced brick and bucket sets (untimed) ------
    tb = torch.zeros(params.brick_capacity, dtype=torch.uint8, device=dev)
    tc = torch.zeros(params.brick_capacity, dtype=torch.uint8, device=dev)
    ts = torch.zeros(params.hash_buckets, dtype=torch.uint8, device=dev)
    tcnt = torch.zeros((H, W, 4), dtype=torch.int32, device=dev)
    traced = dict(out, trace_bricks=tb, trace_color=tc, trace_slots=ts, trace_counts=tcnt)
    bytes_per_pose = []
    n_bd, n_cd, n_sl = [], [], []
    hits = []
    counts = []
    mae = []
    for j, T in enumerate(poses):
        tb.zero_(); tc.zero_(); ts.zero_()
        gm.render(cam, T, out=traced)
        # geometric post-fusion error (Sec. 8): the render at a fused frame's pose against
        # that frame's input depth
        mae.append(dtsdf.depth_error(out["depth"], frames_dev[j][0])[0])
        nb, nc, ns = int(tb.sum()), int(tc.sum()), int(ts.sum())
        n_bd.append(nb); n_cd.append(nc); n_sl.append(ns)
        hits.append(int(out["mask"].sum()))
        # per wave: a single view's work tile takes 16 quads of 2x2 pixels interleaved over a
        # 128x32 region (lane = 16 qy + 4 qx + 2 dy + dx of tile (tx, ty): u = 128 (tx // 16)
        # + 32 qx + 2 (tx % 16) + dx, v = 32 (ty // 4) + 8 qy + 2 (ty % 4) + dy), so the image
        # regroups as (gy, qy, sy, dy, gx, qx, sx, dx) -> waves (gy, sy, gx, sx)
        c = tcnt.view(H // 32, 4, 4, 2, W // 128, 4, 16, 2, 4) \
            .permute(0, 2, 4, 6, 1, 5, 3, 7, 8).reshape(-1, 64, 4).float()
        counts.append(torch.stack([c.mean((0, 1)), c.amax(1).mean(0)]).cpu().numpy())
        bytes_per_pose.append(nb * BRICK_MARCH_BYTES + nc * BRICK_COLOR_BYTES +
                              ns * RECORD_BYTES + H * W * OUT_BYTES_PER_RAY)
    bytes_per_launch = float(np.mean(bytes_per_pose))
    log(f"per pose: bricks {np.mean(n_bd):.0f}, colour bricks {np.mean(n_cd):.0f}, block records "
        f"{np.mean(n_sl):.0f}, hit rate {np.mean(hits) / (H * W):.3f}, "
        f"{bytes_per_launch / 1e6:.2f} MB")
    cnt = np.mean(counts, 0)
    per_ray = dict(zip(["eval", "skip", "absent", "refine"], cnt[0].round(2).tolist()))
    per_wave_max = dict(zip(["eval", "skip", "absent", "refine"], cnt[1].round(2).tolist()))
    log(f"per ray mean {per_ray}; per 8x8 wave, mean of the lane maximum {per_wave_max}")
    log(f"post-fusion depth MAE {np.mean(mae) * 1e3:.3f} mm (mean over the {n} frames)")

    # ---- input preprocessing (Sec. 7): depth filter, normals, normal filter ------------
    pre = dtsdf.Preprocess()
    pev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(50)]
    removed = []
    for j in range(50):
        d_ = frames_dev[j][0]
        pev[j][0].record(stream)
        fd = dtsdf.depth_filter(d_, pre.depth)
        pev[j][1].record(stream)
        _, nn = dtsdf.vertex_normal(fd, cam)
        pev[j][2].record(stream)
        dtsdf.normal_filter(nn, pre.normal_sigma_d, pre.normal_sigma_r_deg, pre.normal_radius)
        pev[j][3].record(stream)
        removed.append(float(((d_ > 0) & (fd == 0)).float().mean()))
    torch.cuda.synchronize()
    preprocess = dict(
        depth_filter_ms=float(np.mean([e[0].elapsed_time(e[1]) for e in pev])),
        vertex_normal_ms=float(np.mean([e[1].elapsed_time(e[2]) for e in pev])),
        normal_filter_ms=float(np.mean([e[2].elapsed_time(e[3]) for e in pev])),
        removed_fraction=float(np.mean(removed)), frames=50,
        params=dataclasses.asdict(pre))
    log(f"preprocess: depth filter {preprocess['depth_filter_ms']:.3f} ms, normals "
        f"{preprocess['vertex_normal_ms']:.3f} ms, normal filter "
        f"{preprocess['normal_filter_ms']:.3f} ms, removed {np.mean(removed):.4f}")
    if not args.no_prefuse:
        # the whole input path of Sec. 7 in fusion: filtered depth, cross-product normals of
        # it, filtered normals steering a second map; post-fusion error of both maps against
        # the raw input depth at every 10th pose
        pm2 = dtsdf.Map(params)
        e0_, e1_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        pre_ms = 0.0
        for k_, (d_, c_) in enumerate(frames_dev):
            e0_.record(stream)
            fd = dtsdf.depth_filter(d_, pre.depth)
            _, nn = dtsdf.vertex_normal(fd, cam)
            nf = dtsdf.normal_filter(nn, pre.normal_sigma_d, pre.normal_sigma_r_deg,
                                     pre.normal_radius)
            pm2.integrate(fd, c_, cam, poses[k_], normal=nf)
            e1_.record(stream)
            e1_.synchronize()
            pre_ms += e0_.elapsed_time(e1_)
        m_raw, m_pre, r_raw, r_pre = [], [], [], []
        for k_ in range(0, n, 10):
            for mp_, errs_, times_ in ((gm, m_raw, r_raw), (pm2, m_pre, r_pre)):
                e0_.record(stream)
                mp_.render(cam, poses[k_], out=out)
                e1_.record(stream)
                errs_.append(dtsdf.depth_error(out["depth"], frames_dev[k_][0])[0])
                e1_.synchronize()
                times_.append(e0_.elapsed_time(e1_))
        preprocess["fusion"] = dict(ms_per_frame=pre_ms / n, bricks=pm2.info()["bricks"],
                                    post_fusion_mae_m=float(np.mean(m_pre)),
                                    plain_post_fusion_mae_m=float(np.mean(m_raw)),
                                    render_ms=float(np.mean(r_pre)),
                                    plain_render_ms=float(np.mean(r_raw)))
        log(f"preprocessed fusion: {pre_ms / n:.3f} ms/frame (filters + integrate), "
            f"{pm2.info()['bricks']} bricks, post-fusion MAE {np.mean(m_pre) * 1e3:.3f} mm vs "
            f"{np.mean(m_raw) * 1e3:.3f} mm plain; render {np.mean(r_pre):.3f} ms vs "
            f"{np.mean(r_raw):.3f} ms")
        del pm2
        torch.cuda.empty_cache()

    if args.copy_probe:
        # a plain elementwise kernel reading and writing 256 MiB each (counter calibration)
        a = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        log(f"copy probe: 3 x (read {a.numel() * 4} B, write {b.numel() * 4} B)")

    # ---- timed render steps ------------------------------------------------------------
    def step(evs=None):
        for j, T in enumerate(poses):
            if evs is not None:
                evs[j][0].record(stream)
            gm.render(cam, T, out=out)
            if evs is not None:
                evs[j][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in poses] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(evs[s])
        log(f"render step {s + 1}/{args.steps} enqueued")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launch_ms = np.array([[a.elapsed_time(b) for (a, b) in e] for e in evs])
    wall = t1 - t0
    rays = args.steps * len(poses) * H * W
    value = rays / wall
    mean_launch_s = float(launch_ms.mean()) * 1e-3
    achieved = bytes_per_launch / mean_launch_s / 1e9
    render_src = os.path.join(ROOT, "paper_2301_12796_amd", "csrc", "render.hip")
    traffic = read_float(read_profile("render_room_640x480_traffic.txt", render_src),
                         "hbm_bytes_per_launch")
    ctr = read_profile("render_room_640x480_counters.txt", render_src)
    valu_per_launch = read_float(ctr, "valu_insts_per_launch")
    valu_frac = (valu_per_launch / (mean_launch_s * VALU_ISSUE_PEAK)
                 if valu_per_launch is not None else None)
    # no-reuse byte model: every evaluation reads the 8 corners (sdf, w) of each present
    # direction of its block from HBM, and every hit the 8 corner colours of each
    d_bar = info["bricks"] / max(info["blocks"], 1)
    evals_per_launch = float(np.mean([c_[0][0] + c_[0][1] + c_[0][3] for c_ in counts])) * H * W
    no_reuse = (evals_per_launch * d_bar * 8 * 8 + float(np.mean(hits)) * d_bar * 8 * 8 +
                H * W * OUT_BYTES_PER_RAY)
    log(f"render roofline: {achieved:.0f} GB/s algorithmic ({achieved / HBM_PEAK_GBS:.4f} of "
        f"HBM peak); VALU issue fraction {valu_frac if valu_frac is None else round(valu_frac, 4)}; "
        f"no-reuse model {no_reuse / 1e9:.2f} GB per launch")

    # ---- cold and warm passes: a view rendered right after 2 GiB of unrelated writes (the
    # caches hold none of the map) and the same view rendered again at once -------------
    flush = torch.empty(1 << 29, dtype=torch.float32, device=dev)
    cold, warm = [], []
    for k_ in range(0, n, max(1, n // 10)):
        e_ = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        flush.fill_(float(k_))
        e_[0].record(stream)
        gm.render(cam, poses[k_], out=out)
        e_[1].record(stream)
        e_[2].record(stream)
        gm.render(cam, poses[k_], out=out)
        e_[3].record(stream)
        torch.cuda.synchronize()
        cold.append(e_[0].elapsed_time(e_[1]))
        warm.append(e_[2].elapsed_time(e_[3]))
    # plain device-to-device copy of 1 GiB (read 1 GiB + write 1 GiB): the HBM rate the box
    # reaches with a streaming kernel
    src_ = flush[: 1 << 28]
    dst_ = torch.empty_like(src_)
    for _ in range(3):
        dst_.copy_(src_)
    ce0, ce1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ce0.record(stream)
    for _ in range(10):
        dst_.copy_(src_)
    ce1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 10 * 2 * src_.numel() * 4 / (ce0.elapsed_time(ce1) * 1e-3) / 1e9
    del flush, src_, dst_
    torch.cuda.empty_cache()
    log(f"cold pass {np.mean(cold):.3f} ms, warm pass {np.mean(warm):.3f} ms; device copy "
        f"{copy_gbs:.0f} GB/s")

    # ---- the same 300 views rendered several per launch (dtsdf_render_batch, the serving
    # form's persistent launch): the tails of the views overlap.  Algorithmic bytes of a
    # launch count the union of the bricks and entries its views touch (traced, untimed) ----
    batched = None
    if args.batch > 1:
        B = args.batch
        groups = [poses[j:j + B] for j in range(0, n, B)]
        bouts = [dict(depth=torch.empty((H, W), dtype=torch.float32, device=dev),
                      normal=torch.empty((3, H, W), dtype=torch.float32, device=dev),
                      rgba=torch.empty((H, W, 4), dtype=torch.uint8, device=dev),
                      mask=torch.empty((H, W), dtype=torch.uint8, device=dev))
                 for _ in range(B)]
        gbytes = []
        for g in groups:
            tb.zero_(); tc.zero_(); ts.zero_()
            tviews = [(cam, T, 0.2, 10.0, dict(bouts[j], trace_bricks=tb, trace_color=tc,
                                               trace_slots=ts)) for j, T in enumerate(g)]
            gm.render_batch(tviews)
            gbytes.append(int(tb.sum()) * BRICK_MARCH_BYTES + int(tc.sum()) * BRICK_COLOR_BYTES +
                          int(ts.sum()) * RECORD_BYTES + len(g) * H * W * OUT_BYTES_PER_RAY)
        views = [[(cam, T, 0.2, 10.0, bouts[j]) for j, T in enumerate(g)] for g in groups]
        for _ in range(args.warmup):
            for vv in views:
                gm.render_batch(vv)
        bev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                for _ in groups] for _ in range(args.steps)]
        torch.cuda.synchronize()
        tb0 = time.perf_counter()
        for s_ in range(args.steps):
            for (e0_, e1_), vv in zip(bev[s_], views):
                e0_.record(stream)
                gm.render_batch(vv)
                e1_.record(stream)
        torch.cuda.synchronize()
        bwall = time.perf_counter() - tb0
        bms = np.array([[a_.elapsed_time(b_) for a_, b_ in e] for e in bev])
        full = [j for j, g in enumerate(groups) if len(g) == B]
        bach = float(np.mean([gbytes[j] for j in full])) / (float(bms[:, full].mean()) * 1e-3) / 1e9
        batched = dict(views_per_launch=B, launches_per_step=len(groups),
                       rays_per_s=n * H * W * args.steps / bwall,
                       ms_per_view=1e3 * bwall / (n * args.steps),
                       roofline=dict(hbm=dict(achieved=bach, peak=HBM_PEAK_GBS, unit="GB/s",
                                              frac=bach / HBM_PEAK_GBS),
                                     algorithmic_bytes_per_launch=float(np.mean([gbytes[j] for j in full])),
                                     mean_launch_ms=float(bms[:, full].mean())))
        log(f"batched ({B} views per launch): {batched['rays_per_s'] / 1e6:.1f} M rays/s, "
            f"{batched['ms_per_view']:.3f} ms per view, {bach:.0f} GB/s algorithmic")

    # ---- precision forms: the same frames fused into f16 / i16 maps ---------------------
    precision = None
    if not args.no_precision:
        precision = {}
        ref = gm.render(cam, poses[150], outputs=("depth", "mask"))
        ref_d = ref["depth"].cpu().numpy()
        for name, sf in (("f16", dtsdf.SDF_F16), ("i16", dtsdf.SDF_I16)):
            pm_ = dtsdf.Map(dtsdf.Params(voxel_size=0.005, truncation=0.02,
                                         brick_capacity=1 << 20, hash_buckets=1 << 21,
                                         sdf_fmt=sf, w_fmt=dtsdf.W_U8))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for k, (d_, c_) in enumerate(frames_dev):
                pm_.integrate(d_, c_, cam, poses[k])
            e1.record(stream)
            torch.cuda.synchronize()
            for T in poses[:10]:
                pm_.render(cam, T, out=out)
            torch.cuda.synchronize()
            pevs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                    for _ in poses]
            for (a_, b_), T in zip(pevs, poses):
                a_.record(stream)
                pm_.render(cam, T, out=out)
                b_.record(stream)
            torch.cuda.synchronize()
            pms = float(np.mean([a_.elapsed_time(b_) for a_, b_ in pevs]))
            q = pm_.render(cam, poses[150], outputs=("depth", "mask"))
            qd = q["depth"].cpu().numpy()
            both = (ref_d > 0) & (qd > 0)
            dz = np.abs(qd - ref_d)[both]
            precision[name] = dict(
                rays_per_s=H * W / (pms * 1e-3), mean_launch_ms=pms,
                integrate_ms_per_frame=e0.elapsed_time(e1) / n,
                device_bytes=pm_.info()["device_bytes"],
                vs_plain_depth_median_m=float(np.median(dz)),
                vs_plain_depth_over_1mm=float(np.mean(dz > 1e-3)),
                vs_plain_depth_over_1cm=float(np.mean(dz > 1e-2)),
                vs_plain_mask_mismatch=float(((ref_d > 0) != (qd > 0)).mean()))
            log(f"precision {name}: {H * W / (pms * 1e-3) / 1e6:.1f} M rays/s, depth vs plain "
                f"median {np.median(dz):.2e} m, over 1 cm {np.mean(dz > 1e-2):.4f}")
            del pm_
            torch.cuda.empty_cache()

    # ---- combined ("rendering") TSDF: recombination, fill and the one-volume render ----
    volume = None
    if not args.no_volume:
        volume = bench_volume(torch, synth, dtsdf, dev, stream, gm, params, cam, poses, out,
                              frames_dev)

    # ---- ICP: three-level point-to-plane SE(3) per frame (10/5/4 iterations) -----------
    icp_ms = icp_dev_ms = icp_rgb_ms = icp_rgb_dev_ms = icp_rgb_err = None
    same = same_rgb = None
    if not args.no_icp:
        icp_frames = list(range(5, n, max(1, n // 10)))[:10]
        tot = tot_dev = 0.0
        same = True
        errs = []
        rng = np.random.default_rng(3)
        for k in icp_frames:
            T = poses[k]
            f = synth.scenes.render_frame(sc, cam, T, noise="quadratic", sigma=0.0012,
                                          seed=9000 + k, device="cuda")
            live = torch.from_numpy(f["depth"]).to(dev)
            dT0 = synth.perturb_pose(0.02, math.radians(2.0), rng)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            levels = []
            for l in range(3):
                c = dtsdf.level_camera(cam, l)
                o = gm.render(c, T, outputs=("vertex", "normal", "mask"))
                levels.append((o["vertex"], o["normal"], o["mask"], c))
            T_est, _ = dtsdf.icp(live, cam, levels, dT0, preprocess=pre)
            torch.cuda.synchronize()
            tot += time.perf_counter() - ta
            errs.append(float(np.linalg.norm(T_est[:3, 3])))
            # the same registration with the model pyramid rendered in one batched launch and
            # every level's iterations enqueued on the device
            torch.cuda.synchronize()
            ta = time.perf_counter()
            levels = dtsdf.render_levels(gm, cam, T)
            T_dev = dtsdf.icp_device(live, cam, levels, dT0, preprocess=pre)
            torch.cuda.synchronize()
            tot_dev += time.perf_counter() - ta
            same = same and bool(np.array_equal(T_dev, T_est))
        icp_ms = 1e3 * tot / len(icp_frames)
        icp_dev_ms = 1e3 * tot_dev / len(icp_frames)
        log(f"icp: {icp_ms:.2f} ms/frame, residual translation median {np.median(errs):.2e} m; "
            f"device loop {icp_dev_ms:.2f} ms/frame, same pose: {same}")
        # combined geometric + photometric ICP against a keyframe (the textured frame of the
        # last multiple of 10, Sec. 5.3), three levels, same offsets
        tot_rgb, tot_rgb_dev, errs_rgb, same_rgb = 0.0, 0.0, [], True
        rng = np.random.default_rng(3)
        for k in icp_frames:
            T = poses[k]
            kf = 10 * (k // 10) if k % 10 else max(0, k - 10)
            T_kf = poses[kf]
            f = synth.scenes.render_frame(sc, cam, T, noise="quadratic", sigma=0.0012,
                                          seed=9000 + k, device="cuda", texture_period=0.25)
            fk = synth.scenes.render_frame(sc, cam, T_kf, device="cuda", texture_period=0.25)
            live = torch.from_numpy(f["depth"]).to(dev)
            live_rgb = torch.from_numpy(f["rgb"]).to(dev)
            kf_rgb = torch.from_numpy(fk["rgb"]).to(dev)
            dT0 = synth.perturb_pose(0.02, math.radians(2.0), rng)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            levels, refs = [], []
            ri = dtsdf.intensity(kf_rgb)
            for l in range(3):
                c = dtsdf.level_camera(cam, l)
                o = gm.render(c, T, outputs=("vertex", "normal", "mask"))
                levels.append((o["vertex"], o["normal"], o["mask"], c))
                refs.append((ri, c))
                if l < 2:
                    ri = dtsdf.intensity_downsample(ri)
            T_est, _ = dtsdf.icp(live, cam, levels, dT0, live_rgb=live_rgb, ref_levels=refs,
                                 T_ref_model=np.linalg.inv(T_kf) @ T, preprocess=pre)
            torch.cuda.synchronize()
            tot_rgb += time.perf_counter() - ta
            errs_rgb.append(float(np.linalg.norm(T_est[:3, 3])))
            # the fast path: model pyramid in one batched launch, iterations on the device
            torch.cuda.synchronize()
            ta = time.perf_counter()
            ri = dtsdf.intensity(kf_rgb)
            refs = []
            for l in range(3):
                refs.append((ri, dtsdf.level_camera(cam, l)))
                if l < 2:
                    ri = dtsdf.intensity_downsample(ri)
            levels = dtsdf.render_levels(gm, cam, T)
            T_dev = dtsdf.icp_device(live, cam, levels, dT0, live_rgb=live_rgb, ref_levels=refs,
                                     T_ref_model=np.linalg.inv(T_kf) @ T, preprocess=pre)
            torch.cuda.synchronize()
            tot_rgb_dev += time.perf_counter() - ta
            same_rgb = same_rgb and bool(np.array_equal(T_dev, T_est))
        icp_rgb_ms = 1e3 * tot_rgb / len(icp_frames)
        icp_rgb_dev_ms = 1e3 * tot_rgb_dev / len(icp_frames)
        icp_rgb_err = float(np.median(errs_rgb))
        log(f"combined icp (keyframe): {icp_rgb_ms:.2f} ms/frame, residual translation "
            f"median {icp_rgb_err:.2e} m; fast path {icp_rgb_dev_ms:.2f} ms/frame, same pose: "
            f"{same_rgb}")

    # ---- multi-sensor Sim(3) refinement: five sensors with scaled depth, taking turns
    # frame by frame, each frame registered by Levenberg-Marquardt Sim(3) ICP (10/5/4) from a
    # nominal calibration 1 % off; scales anchored to sensor 0 (Sec. 6, Sec. 7) ------------
    multi = None
    if not args.no_icp:
        scales = (1.0, 1.05, 0.975, 1.025, 0.95)
        rng = np.random.default_rng(5)
        tot, logs = 0.0, {i: [] for i in range(5)}
        lm_frames = list(range(3, n, max(1, n // 20)))[:20]
        for j, k in enumerate(lm_frames):
            i = j % 5
            T = poses[k]
            f = synth.scenes.render_frame(sc, cam, T, noise="quadratic", sigma=0.0012,
                                          seed=7000 + k, device="cuda", depth_scale=scales[i])
            live = torch.from_numpy(f["depth"]).to(dev)
            dT0 = synth.perturb_pose(0.01, math.radians(1.0), rng)
            dT0[:3, :3] *= 1.01 / scales[i]
            torch.cuda.synchronize()
            ta = time.perf_counter()
            levels = dtsdf.render_levels(gm, cam, T)      # model pyramid in one launch
            T_est, _ = dtsdf.icp_lm(live, cam, levels, dT0, dim=7, preprocess=pre)
            torch.cuda.synchronize()
            tot += time.perf_counter() - ta
            logs[i].append(math.log(float(np.cbrt(np.linalg.det(T_est[:3, :3])))))
        raw = [float(np.mean(logs[i])) for i in range(5)]
        anchored = [r - raw[0] for r in raw]
        err = [abs(a - math.log(scales[0] / s_)) for a, s_ in zip(anchored, scales)]
        multi = dict(sensors=list(scales), frames=len(lm_frames),
                     lm_sim3_ms_per_frame=1e3 * tot / len(lm_frames),
                     raw_log_scale=raw, anchored_log_scale=anchored,
                     anchored_log_scale_error_max=float(max(err)))
        log(f"multi-sensor LM Sim(3): {multi['lm_sim3_ms_per_frame']:.2f} ms/frame, anchored "
            f"log-scale error max {max(err):.2e}")

    # ---- map upkeep (Sec. 3): recycling of bricks without surface, on the fused map; the
    # render and the post-fusion error at every 10th pose before and after ---------------
    upkeep = None
    if not args.no_recycle:
        sub = list(range(0, n, 10))

        def render_pass():
            evs_ = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                    for _ in sub]
            errs = []
            for (a_, b_), k in zip(evs_, sub):
                a_.record(stream)
                gm.render(cam, poses[k], out=out)
                b_.record(stream)
                errs.append(dtsdf.depth_error(out["depth"], frames_dev[k][0])[0])
            torch.cuda.synchronize()
            return float(np.mean([a_.elapsed_time(b_) for a_, b_ in evs_])), float(np.mean(errs))

        ms0, mae0 = render_pass()
        upkeep = dict(bricks_before=gm.info()["bricks"], render_ms_before=ms0,
                      post_fusion_mae_before_m=mae0, passes=[])
        for t_free in (0.9, 0.5):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            nrec = gm.recycle(t_free)
            dt = time.perf_counter() - ta
            ms1, mae1 = render_pass()
            upkeep["passes"].append(dict(t_free=t_free, recycled=nrec, recycle_ms=1e3 * dt,
                                         bricks_after=gm.info()["bricks"], render_ms=ms1,
                                         post_fusion_mae_m=mae1))
            log(f"recycle t_free={t_free}: {nrec} bricks in {1e3 * dt:.2f} ms, render "
                f"{ms0:.3f} -> {ms1:.3f} ms, post-fusion MAE {mae0 * 1e3:.3f} -> "
                f"{mae1 * 1e3:.3f} mm")

    # ---- tracking: 640x480 live frames against the tiny map -----------------------------
    tracking = None
    if not args.no_icp:
        tracking = bench_tracking(torch, synth, dtsdf, dev)

    # ---- serving: render + Sim(3) ICP requests from four sensors on the tiny map -------
    serving = None
    if not args.no_serve:
        serving = bench_serving(args, torch, synth, dtsdf, dev)

    # ---- CPU baseline: the FP64 oracle on a bounded sample -----------------------------
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as orc
        om = orc.OracleMap(orc.MapParams(voxel=0.005, tau=0.02))
        # every tenth of the fused frames (the oracle fuses a frame in about a second)
        sample_frames = list(range(0, n, 10))
        ta_ = time.perf_counter()
        for k in sample_frames:
            f = synth.scenes.render_frame(sc, cam, synth.room_pose(k, n), noise="quadratic",
                                          sigma=0.0012, seed=2000 + k, z_max=10.0,
                                          device="cuda")
            om.integrate(f["depth"], f["rgb"], cam, synth.room_pose(k, n))
        t_fuse = time.perf_counter() - ta_
        log(f"cpu baseline: oracle map fused from {len(sample_frames)} frames in {t_fuse:.1f} s, "
            f"{om.num_bricks} bricks (GPU map {info['bricks']})")
        # whole frames of consecutive trajectory poses from pose 30 on, 8 rows at a time,
        # until cpu_seconds of oracle time have been spent
        rays_done, t_cpu, pose_k, rows_done = 0, 0.0, 30, 0
        while t_cpu < args.cpu_seconds:
            vv, uu = np.mgrid[rows_done:rows_done + 8, 0:W]
            pix = np.stack([uu.ravel(), vv.ravel()], 1)
            ta = time.perf_counter()
            om.render(cam, poses[pose_k % n], pixels=pix, classify=False)
            t_cpu += time.perf_counter() - ta
            rays_done += pix.shape[0]
            rows_done += 8
            if rows_done >= H:
                rows_done, pose_k = 0, pose_k + 1
        frames_txt = f"{rays_done / (H * W):.2f} frames from trajectory pose 30 on"
        cpu = dict(value=rays_done / t_cpu, unit="rays/s", cores=orc.num_threads(),
                   kind="oracle",
                   sample=f"FP64 oracle render (depth+normal+colour) of {frames_txt} "
                          f"({rays_done} rays, {t_cpu:.1f} s) on an oracle map fused from "
                          f"every tenth of the {n} frames ({len(sample_frames)} frames, "
                          f"{om.num_bricks} bricks; the GPU map holds all {n}, "
                          f"{info['bricks']} bricks)")
        log(f"cpu baseline: {cpu['value']:.0f} rays/s on {cpu['cores']} threads")

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "room 4x4x3 m, seeded boxes/spheres/5 mm plates, 300 frames 640x480 "
                        "fused at 5 mm voxels, tau 2 cm; render depth+normal+colour at the "
                        "300 trajectory poses per step",
            "width": W, "height": H, "poses_per_step": len(poses), "voxel_m": 0.005,
            "truncation_m": 0.02, "bricks": info["bricks"], "blocks": info["blocks"],
        },
        "roofline": roofline_block(achieved, traffic, valu_per_launch, valu_frac,
                                   mean_launch_s, ctr) | {
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "mean_launch_ms": float(launch_ms.mean()),
            "bricks_per_launch": float(np.mean(n_bd)),
            "color_bricks_per_launch": float(np.mean(n_cd)),
            "block_records_per_launch": float(np.mean(n_sl)),
            "no_reuse_bytes_per_launch": no_reuse,
            "cold_pass_ms": float(np.mean(cold)),
            "warm_pass_ms": float(np.mean(warm)),
            "device_copy_gbs": copy_gbs,
            "frac_of_device_copy": achieved / copy_gbs,
        },
        "cpu_baseline": cpu,
        "integrate_ms_per_frame": integ_ms / n,
        "fusion": fusion,
        "icp_ms_per_frame": icp_ms,
        "icp_device_loop_ms_per_frame": icp_dev_ms,
        "icp_device_loop_same_pose": same,
        "icp_rgb_keyframe_ms_per_frame": icp_rgb_ms,
        "icp_rgb_keyframe_device_loop_ms_per_frame": icp_rgb_dev_ms,
        "icp_rgb_keyframe_device_loop_same_pose": same_rgb,
        "icp_rgb_keyframe_translation_median_m": icp_rgb_err,
        "batched": batched,
        "multi_sensor": multi,
        "post_fusion_mae_m": float(np.mean(mae)),
        "upkeep": upkeep,
        "preprocess": preprocess,
        "hit_rate": float(np.mean(hits) / (H * W)),
        "samples_per_ray": per_ray,
        "samples_per_wave_max": per_wave_max,
        "input_generation_s": t_gen,
        "tracking": tracking,
        "serving": serving,
        "precision": precision,
        "volume": volume,
    }
    print(json.dumps(line), flush=True)


def bench_volume(torch, synth, dtsdf, dev, stream, gm, params, cam, poses, out, frames_dev):
    """The view-dependent combined TSDF on the room map: a full recombination (frustum
    widened by 1/8) per trajectory pose, the render of the resulting volume from that pose
    against the direct six-direction render, and a frame loop in which every frame is fused,
    the conditional-recombination policy (boot up 5, stale 50 frames, 5 cm, 0.05 pi/2 rad)
    decides between a recombination and a fill of the voxels seen for the first time, and
    the volume is rendered at the frame's pose.  Frames 100 .. 159 are first registered
    (three-level ICP, preprocessed live frame, 2 cm / 2 degree offsets; model pyramid in one
    batched launch, iterations enqueued on the device) against renders of the volume and,
    for comparison, of the map.  Timings include the model renders, not the
    recombination."""
    H, W = cam.height, cam.width
    ev = lambda: torch.cuda.Event(enable_timing=True)
    vol = dtsdf.Volume(gm, brick_capacity=1 << 18, hash_buckets=1 << 18)
    vol.combine(gm, cam, poses[0])          # first call gives every block its brick
    torch.cuda.synchronize()
    comb_ms, rend_ms = [], []
    for T in poses:
        a_, b_, c_ = ev(), ev(), ev()
        a_.record(stream)
        vol.combine(gm, cam, T)
        b_.record(stream)
        vol.render(cam, T, out=out)
        c_.record(stream)
        c_.synchronize()
        comb_ms.append(a_.elapsed_time(b_))
        rend_ms.append(b_.elapsed_time(c_))
    # algorithmic bytes of the volume render (traced brick / bucket sets, as for the direct
    # render) and accuracy against the direct render, at 10 poses
    vcap = 1 << 18
    tb = torch.zeros(vcap, dtype=torch.uint8, device=dev)
    tc = torch.zeros(vcap, dtype=torch.uint8, device=dev)
    ts = torch.zeros(1 << 18, dtype=torch.uint8, device=dev)
    vbytes = []
    dz_all, mm, one = [], [], []
    for T in poses[::30]:
        vol.combine(gm, cam, T)
        tb.zero_(); tc.zero_(); ts.zero_()
        vol.render(cam, T, out=dict(out, trace_bricks=tb, trace_color=tc, trace_slots=ts))
        vbytes.append(int(tb.sum()) * BRICK_MARCH_BYTES + int(tc.sum()) * BRICK_COLOR_BYTES +
                      int(ts.sum()) * RECORD_BYTES + H * W * OUT_BYTES_PER_RAY)
        v = vol.render(cam, T, outputs=("depth", "mask"))
        d = gm.render(cam, T, outputs=("depth", "mask"))
        vd, dd = v["depth"].cpu().numpy(), d["depth"].cpu().numpy()
        both = (vd > 0) & (dd > 0)
        dz_all.append(np.abs(vd - dd)[both])
        mm.append(float(((vd > 0) != (dd > 0)).mean()))
    dz = np.concatenate(dz_all)
    vinfo = vol.info()
    del vol
    # frame loop with conditional recombination on a map fused frame by frame
    fm = dtsdf.Map(params)
    fv = dtsdf.Volume(fm, brick_capacity=1 << 18, hash_buckets=1 << 18)
    pol = dtsdf.RecombinePolicy()
    n_re, loop_ms, direct_ms = 0, [], []
    last = None
    # tracking inside the loop (frames 100 .. 159, before each is fused): three-level ICP of
    # the frame against renders of the combined volume and, separately, of the map itself
    track = dict(volume_ms=[], direct_ms=[], volume_err=[], direct_err=[])
    rng = np.random.default_rng(17)
    pre = dtsdf.Preprocess()
    for k, (d_, c_) in enumerate(frames_dev):
        T = poses[k]
        if 100 <= k < 160 and last is not None:
            dT0 = synth.perturb_pose(0.02, math.radians(2.0), rng)
            for name, src in (("volume", fv), ("direct", fm)):
                torch.cuda.synchronize()
                ta = time.perf_counter()
                levels = dtsdf.render_levels(src, cam, T)
                T_est = dtsdf.icp_device(d_, cam, levels, dT0, preprocess=pre)
                torch.cuda.synchronize()
                track[name + "_ms"].append(1e3 * (time.perf_counter() - ta))
                track[name + "_err"].append(float(np.linalg.norm(T_est[:3, 3])))
        fm.integrate(d_, c_, cam, T)
        torch.cuda.synchronize()
        a_, b_ = ev(), ev()
        a_.record(stream)
        if pol.decide(T):
            fv.combine(fm, cam, T)
            last = T
            n_re += 1
        else:
            fv.combine(fm, cam, last, T_frustum=T, margin=0.0, only_missing=True)
        fv.render(cam, T, out=out)
        b_.record(stream)
        b_.synchronize()
        loop_ms.append(a_.elapsed_time(b_))
        if k % 10 == 0:
            c0, c1 = ev(), ev()
            c0.record(stream)
            fm.render(cam, T, out=out)
            c1.record(stream)
            c1.synchronize()
            direct_ms.append(c0.elapsed_time(c1))
    del fv, fm
    torch.cuda.empty_cache()
    res = dict(
        combine_ms=float(np.mean(comb_ms)), combine_ms_max=float(np.max(comb_ms)),
        render_ms=float(np.mean(rend_ms)), render_rays_per_s=H * W / (np.mean(rend_ms) * 1e-3),
        render_algorithmic_bytes=float(np.mean(vbytes)),
        render_achieved_gbs=float(np.mean(vbytes)) / (np.mean(rend_ms) * 1e-3) / 1e9,
        vs_direct_depth_median_m=float(np.median(dz)),
        vs_direct_depth_over_1mm=float(np.mean(dz > 1e-3)),
        vs_direct_depth_over_1cm=float(np.mean(dz > 1e-2)),
        vs_direct_mask_mismatch=float(np.mean(mm)),
        volume_device_bytes=vinfo["device_bytes"], volume_blocks=vinfo["blocks"],
        loop_frames=len(frames_dev), loop_recombined=n_re,
        loop_ms_per_frame=float(np.mean(loop_ms)),
        loop_direct_render_ms=float(np.mean(direct_ms)),
        tracking=dict(frames=len(track["volume_ms"]),
                      volume_icp_ms_per_frame=float(np.mean(track["volume_ms"])),
                      direct_icp_ms_per_frame=float(np.mean(track["direct_ms"])),
                      volume_translation_median_m=float(np.median(track["volume_err"])),
                      direct_translation_median_m=float(np.median(track["direct_err"]))))
    log(f"volume: combine {res['combine_ms']:.2f} ms, render {res['render_ms']:.2f} ms "
        f"({res['render_rays_per_s'] / 1e6:.1f} M rays/s), depth vs direct median "
        f"{res['vs_direct_depth_median_m']:.2e} m, >1 cm {res['vs_direct_depth_over_1cm']:.4f}, "
        f"mask mismatch {res['vs_direct_mask_mismatch']:.4f}; loop: {n_re}/{len(frames_dev)} "
        f"recombined, {res['loop_ms_per_frame']:.2f} ms/frame (combine or fill + render) vs "
        f"direct render {res['loop_direct_render_ms']:.2f} ms")
    tr_ = res["tracking"]
    log(f"tracking against the volume: {tr_['volume_icp_ms_per_frame']:.2f} ms/frame, residual "
        f"{tr_['volume_translation_median_m']:.2e} m; against the map: "
        f"{tr_['direct_icp_ms_per_frame']:.2f} ms/frame, {tr_['direct_translation_median_m']:.2e} m")
    return res


def tiny_map(torch, synth, dtsdf, dev):
    """The tiny-scene map: dense 64^3 blocks at 1 cm (tau 4 cm) fused from its ten frames."""
    tm = dtsdf.Map(dtsdf.Params(voxel_size=0.01, truncation=0.04, brick_capacity=4096,
                                hash_buckets=1 << 12, dense_lo=synth.scenes.TINY_DENSE_LO,
                                dense_hi=synth.scenes.TINY_DENSE_HI))
    for f in synth.tiny_frames(10):
        tm.integrate(torch.from_numpy(f["depth"]).to(dev), torch.from_numpy(f["rgb"]).to(dev),
                     synth.scenes.TINY_CAMERA, f["T_wc"])
    return tm


def bench_tracking(torch, synth, dtsdf, dev):
    """The tracking workload: live 640x480 frames (f = 525, depth noise 0.5 mm) of the tiny
    scene at 30 seeded poses of its circle, registered against the tiny map from 2 cm /
    2 degree offsets by three-level point-to-plane ICP (10/5/4 iterations).  Per frame: the
    model pyramid rendered in one batched launch, then the ICP with a host wait per
    iteration (icp) and with every level's iterations enqueued on the device (icp_device).
    Reports ms/frame, the pose error against the truth (the live frame is taken at the model
    pose, so the result should be the identity) and cond(H) of each level's last step."""
    tm = tiny_map(torch, synth, dtsdf, dev)
    cam = synth.scenes.Camera(640, 480, 525.0, 525.0, 319.5, 239.5)
    sc = synth.tiny_scene()
    cases = synth.tracking_cases(30)
    lives = [torch.from_numpy(synth.render_frame(sc, cam, T, noise="const", sigma=0.0005,
                                                 seed=7000 + i, device="cuda")["depth"]).to(dev)
             for i, (T, _) in enumerate(cases)]
    for (T, dT0), live in list(zip(cases, lives))[:3]:                  # warm-up
        dtsdf.icp(live, cam, dtsdf.render_levels(tm, cam, T, z_far=2.5), dT0)
    torch.cuda.synchronize()
    rot, trans, conds, t_host, t_dev, same = [], [], [], 0.0, 0.0, True
    for (T, dT0), live in zip(cases, lives):
        ta = time.perf_counter()
        levels = dtsdf.render_levels(tm, cam, T, z_far=2.5)
        T_est, lg = dtsdf.icp(live, cam, levels, dT0)
        torch.cuda.synchronize()
        t_host += time.perf_counter() - ta
        ta = time.perf_counter()
        levels = dtsdf.render_levels(tm, cam, T, z_far=2.5)
        T_dev = dtsdf.icp_device(live, cam, levels, dT0)
        torch.cuda.synchronize()
        t_dev += time.perf_counter() - ta
        same = same and bool(np.array_equal(T_dev, T_est))
        c = np.clip((np.trace(T_est[:3, :3]) - 1.0) / 2.0, -1.0, 1.0)
        rot.append(float(np.arccos(c)))
        trans.append(float(np.linalg.norm(T_est[:3, 3])))
        last = {}
        for e in lg:
            if "H" in e:
                last[e["level"]] = e["H"]
        conds.append([float(np.linalg.cond(last[l])) if l in last else float("nan")
                      for l in range(3)])
    conds = np.array(conds)
    out = dict(cases=len(cases), ms_per_frame=1e3 * t_host / len(cases),
               device_loop_ms_per_frame=1e3 * t_dev / len(cases), device_loop_same_pose=same,
               rot_error_median_rad=float(np.median(rot)), rot_error_max_rad=float(np.max(rot)),
               trans_error_median_m=float(np.median(trans)),
               trans_error_max_m=float(np.max(trans)),
               cond_H_median_per_level=[float(np.nanmedian(conds[:, l])) for l in range(3)],
               cond_H_max_per_level=[float(np.nanmax(conds[:, l])) for l in range(3)])
    log(f"tracking (tiny scene, 30 cases): {out['ms_per_frame']:.2f} ms/frame "
        f"({out['device_loop_ms_per_frame']:.2f} device loop, same pose {same}); error vs truth "
        f"rot median {out['rot_error_median_rad']:.2e} rad, trans median "
        f"{out['trans_error_median_m']:.2e} m; cond(H) median per level "
        f"{[round(c_, 0) for c_ in out['cond_H_median_per_level']]}")
    return out


def bench_serving(args, torch, synth, dtsdf, dev):
    """The serving workload: the tiny-scene map resident (dense 64^3 blocks at 1 cm, fused
    from its 10 frames), four sensors (320x240 .. 1280x720, seeded intrinsics and depth
    scale factors), a Poisson stream of 3600 requests at 120 requests/s; each request is a
    three-level model render plus 10/5/4 Sim(3) ICP iterations from a 2 cm / 2 degree / 1 %
    prior.  Reports arrival -> pose latency of the continuous-batching server (32 slots,
    request buffers carved from an arena of 1 % of the device memory free at start-up) and
    of serial unbatched calls, at 120 req/s and, with the same requests on a compressed
    timeline, at 480 and 1000 req/s (the serial baseline on the first 600 requests there);
    and the capacity of both with every request queued at the start."""
    from paper_2301_12796_amd import serve
    tm = tiny_map(torch, synth, dtsdf, dev)
    sensors = synth.serving_sensors()
    t = time.time()
    work = synth.serving_workload(args.serve_requests, device="cuda")
    depths = [torch.from_numpy(w["depth"]).to(dev) for w in work]
    torch.cuda.synchronize()
    log(f"serving: {len(work)} requests generated in {time.time() - t:.1f} s, last arrival "
        f"{work[-1]['arrival']:.2f} s")
    px = [sum((sensors[w["sensor"]][0].width >> l) * (sensors[w["sensor"]][0].height >> l)
              for l in range(3)) for w in work]

    def reqs(rate=120.0, n=None):
        k_ = len(work) if n is None else min(n, len(work))
        return [serve.Request(k, w["arrival"] * 120.0 / rate, w["sensor"], depths[k],
                              w["T_model"], w["dT0"]) for k, w in enumerate(work[:k_])]

    serve.Server(tm, sensors).run(reqs()[:16], realtime=False)        # warm-up
    serve.serve_serial(tm, sensors, reqs()[:4], realtime=False)
    torch.cuda.synchronize()
    sweep = []
    done120 = ser120 = None
    for rate in (120.0, 480.0, 1000.0):
        srv = serve.Server(tm, sensors)
        t0 = time.perf_counter()
        done = srv.run(reqs(rate), realtime=True)
        wall = time.perf_counter() - t0
        lat = serve.latency_stats(done)
        n_ser = len(work) if rate == 120.0 else min(600, len(work))
        ser = serve.serve_serial(tm, sensors, reqs(rate, n_ser), realtime=True)
        lat_s = serve.latency_stats(ser)
        row = dict(rate_per_s=rate, requests=len(done), p50_ms=lat["p50_ms"],
                   p99_ms=lat["p99_ms"], mean_batch=float(np.mean(srv.batch_sizes)),
                   max_batch=int(max(srv.batch_sizes)), rays_per_s=sum(px) / wall,
                   peak_arena_bytes=int(srv.peak_bytes), arena_bytes=int(srv.budget),
                   admissions_deferred=int(srv.deferred), serial_requests=n_ser,
                   serial_p50_ms=lat_s["p50_ms"], serial_p99_ms=lat_s["p99_ms"])
        sweep.append(row)
        log(f"served at {rate:.0f} req/s: p50 {lat['p50_ms']:.2f} ms, p99 {lat['p99_ms']:.2f} ms, "
            f"mean batch {row['mean_batch']:.2f} (max {row['max_batch']}); serial ({n_ser}): "
            f"p50 {lat_s['p50_ms']:.2f} ms, p99 {lat_s['p99_ms']:.2f} ms")
        if rate == 120.0:
            done120, ser120 = done, ser
    bitwise = all(np.array_equal(a.pose, b.pose) for a, b in
                  zip(sorted(done120, key=lambda r: r.rid), sorted(ser120, key=lambda r: r.rid)))
    srv2 = serve.Server(tm, sensors)
    t0 = time.perf_counter()
    srv2.run(reqs(), realtime=False)
    cap = len(work) / (time.perf_counter() - t0)
    n_cap = min(600, len(work))
    t0 = time.perf_counter()
    serve.serve_serial(tm, sensors, reqs(120.0, n_cap), realtime=False)
    cap_s = n_cap / (time.perf_counter() - t0)
    log(f"capacity: batched {cap:.0f} req/s, serial {cap_s:.0f} req/s; alone == mix: {bitwise}")
    scale_err = [abs(np.cbrt(np.linalg.det(r.pose[:3, :3])) * work[r.rid]["scale"] - 1.0)
                 for r in done120]
    base = sweep[0]
    return dict(requests=len(work), rate_per_s=120.0, slots=srv2.slots_count,
                p50_ms=base["p50_ms"], p99_ms=base["p99_ms"],
                serial_p50_ms=base["serial_p50_ms"], serial_p99_ms=base["serial_p99_ms"],
                rays_per_s=base["rays_per_s"], mean_batch=base["mean_batch"],
                capacity_req_per_s=cap, serial_capacity_req_per_s=cap_s,
                serial_capacity_sample=f"first {n_cap} requests",
                alone_vs_mix_bitwise=bool(bitwise),
                scale_error_median=float(np.median(scale_err)),
                arena_bytes=int(srv2.budget), rate_sweep=sweep,
                sample=f"all {len(work)} requests of the stream")


if __name__ == "__main__":
    main()
