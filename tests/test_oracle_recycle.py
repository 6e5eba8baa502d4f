"""Pins of the oracle's brick recycling (Sec. 3: bricks that repeated carving turned into
free space go back to the pool).

* hand-built bricks: never observed -> removed; every observed value >= t_free -> removed,
  also at equality and when a lower value sits in an unobserved voxel; one observed value
  below t_free -> kept, contents untouched;
* an object removed from the scene: after carving (carving weight 1), recycling at
  t_free = 0.5 (2 cm, two voxels, from any surface, so no cell next to a freed voxel can
  hold a crossing of a consistent field) frees most of its bricks and keeps every brick with
  a surface value; the render changes only where a remnant of the object hid the scene, and
  there it moves to the scene as it is now.
"""
import numpy as np

import synth
from synth.scenes import Box, Camera, Room, Scene, Sphere, look_at, render_frame
from oracle import oracle as O


def _blob(bricks):
    n = len(bricks)
    keys = np.array([[i, 0, 0, 0] for i in range(n)], np.int32)
    sdf = np.stack([b[0] for b in bricks]).astype(np.float32)
    w = np.stack([b[1] for b in bricks]).astype(np.float32)
    return dict(keys=keys, sdf=sdf, w=w, rgb=np.zeros((n, 512, 3), np.uint8),
                wc=np.zeros((n, 512), np.float32))


def test_recycle_definition_on_hand_built_bricks():
    one, zero = np.ones(512), np.zeros(512)
    low = np.full(512, 0.95)
    low[7] = 0.2
    hidden = low.copy()
    w_hidden = one.copy()
    w_hidden[7] = 0.0
    bricks = [(zero, zero),                  # 0 never observed           -> removed
              (np.full(512, 0.95), one),     # 1 free space                -> removed
              (low, one),                    # 2 one surface value         -> kept
              (np.full(512, 0.5), one),      # 3 exactly t_free            -> removed
              (hidden, w_hidden)]            # 4 low value not observed    -> removed
    m = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04))
    m.load(_blob(bricks))
    assert m.recycle(0.5) == 4
    out = m.export()
    assert out["keys"].tolist() == [[2, 0, 0, 0]]
    np.testing.assert_array_equal(out["sdf"][0], low.astype(np.float32))
    assert m.recycle(0.5) == 0


def _scenes():
    room = Room(np.array([-2.0, -2.0, -1.5]), np.array([2.0, 2.0, 1.5]),
                np.tile(np.array([90, 90, 90], np.uint8), (6, 1)))
    plate = Box(np.array([0.295, -0.30, -0.30]), np.array([0.305, 0.30, 0.30]),
                np.tile(np.array([120, 120, 120], np.uint8), (6, 1)))
    ball = Sphere(np.array([-0.1, 0.1, 0.0]), 0.15, np.array([210, 90, 50], np.uint8))
    return Scene(spheres=[ball], boxes=[plate], room=room), \
        Scene(spheres=[], boxes=[plate], room=room)


def carving_workload(n_with=4, n_without=10):
    """Frames of a scene with a ball, then frames of the same scene without it."""
    cam = Camera(160, 120, 120.0, 120.0, 79.5, 59.5)
    with_ball, without = _scenes()
    poses = synth.tiny_cameras(n_with + n_without, seed=5)
    frames = []
    for k, T in enumerate(poses):
        sc = with_ball if k < n_with else without
        f = render_frame(sc, cam, T, noise="const", sigma=0.0005, seed=500 + k, z_max=10.0)
        f["T_wc"] = T
        frames.append(f)
    return cam, frames


def test_removed_object_is_recycled_and_only_its_remnants_leave_the_render():
    cam, frames = carving_workload()
    m = O.OracleMap(O.MapParams(voxel=0.01, tau=0.04, w_carve=1.0))
    for f in frames:
        m.integrate(f["depth"], f["rgb"], cam, f["T_wc"])
    before = m.export()
    T = look_at((0.9, -0.4, 0.1), (0.0, 0.0, 0.0))
    r0 = m.render(cam, T, classify=False)
    n0 = len(before["keys"])
    removed = m.recycle(0.5)
    after = m.export()
    r1 = m.render(cam, T, classify=False)
    # bricks of the ball (within 2 cm of its surface and away from the plate and walls)
    centers = (before["keys"][:, :3] + 0.5) * 0.08
    dist_ball = np.abs(np.linalg.norm(centers - np.array([-0.1, 0.1, 0.0]), axis=1) - 0.15)
    kept = set(map(tuple, after["keys"]))
    ball_only = [tuple(k) for k, d in zip(before["keys"], dist_ball)
                 if d < 0.02 and abs(k[0] * 0.08 + 0.04 - 0.3) > 0.15]
    gone = sum(k not in kept for k in ball_only)
    print(f"bricks {n0} -> {len(after['keys'])}, removed {removed}; ball bricks "
          f"{len(ball_only)}, recycled {gone}")
    assert len(ball_only) > 50 and gone > 0.8 * len(ball_only) and removed >= gone
    # every brick still holding an observed value below t_free stays
    obs_low = ((before["w"] > 0) & (before["sdf"] < np.float32(0.5))).any(1)
    assert set(map(tuple, before["keys"][obs_low])) == kept
    # the render changes only where a remnant of the ball (a crossing next to a freed brick)
    # hid the scene as it is now, and every change moves towards the true depth
    true = render_frame(_scenes()[1], cam, T)["true_depth"].ravel()
    hit0, hit1 = r0.mask > 0, r1.mask > 0
    assert (hit0 != hit1).mean() < 1e-3
    both = hit0 & hit1 & (true > 0)
    changed = both & (r0.depth != r1.depth)
    e0, e1 = np.abs(r0.depth - true), np.abs(r1.depth - true)
    print(f"changed pixels {int(changed.sum())}, error there {np.median(e0[changed]):.3f} -> "
          f"{np.median(e1[changed]):.4f} m")
    assert changed.mean() < 0.01
    assert np.all(e1[changed] <= e0[changed])
    assert np.all(e1[both & ~changed] == e0[both & ~changed])
