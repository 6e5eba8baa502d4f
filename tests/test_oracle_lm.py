"""Pins of the oracle's Levenberg-Marquardt solver with Madsen's damping (Sec. 7) and of
scale anchoring (Sec. 6, eq. scale_anchor).

* the damping core minimises Rosenbrock's function written as least squares, a textbook
  test problem with the known minimum (1, 1), with a monotone cost over accepted steps;
* with tau = 0 (no damping) every step of a well-posed registration is accepted and the
  iterates are those of Gauss-Newton;
* LM Sim(3) ICP recovers a depth scale exactly on a noise-free scene (exp(sigma) = 1/s);
* anchoring removes a drift common to all sensors' log-scale estimates.
"""
import math

import numpy as np
import pytest

import synth
from synth.scenes import Camera, render_frame
from oracle import oracle as O
from tests.test_oracle_pins import _box_world, _model_levels


def test_damping_core_minimises_rosenbrock():
    def f(x):
        return np.array([10.0 * (x[1] - x[0] ** 2), 1.0 - x[0]])

    def J(x):
        return np.array([[-20.0 * x[0], 10.0], [-1.0, 0.0]])

    st = O.LmState(tau=1e-3)
    x = np.array([-1.2, 1.0])
    cand = x.copy()
    costs = []
    for _ in range(200):
        r, Jr = f(cand), J(cand)
        # residual convention of the ICP sums: H = J^T J, g = J^T r, F = sum r^2
        if O.lm_update(st, Jr.T @ Jr, Jr.T @ r, float(r @ r)):
            x = cand
            costs.append(float(r @ r))
        h = O.lm_step(st)
        cand = x + h
        if np.linalg.norm(h) < 1e-14:
            break
    assert np.max(np.abs(x - 1.0)) < 1e-8
    assert all(b <= a for a, b in zip(costs, costs[1:]))
    assert len(costs) > 5


def test_undamped_lm_is_gauss_newton():
    sc = _box_world()
    cam = Camera(640, 480, 525.0, 525.0, 319.5, 239.5)
    T = synth.room_pose(40)
    live = render_frame(sc, cam, T)["depth"]
    dT0 = synth.perturb_pose(0.01, math.radians(1.0), np.random.default_rng(6))
    levels = _model_levels(sc, cam, T)
    T_gn, log_gn = O.icp(live, cam, levels, dT0, dim=6)
    T_lm, log_lm = O.icp_lm(live, cam, levels, dT0, dim=6, tau=0.0)
    assert all(e["accepted"] for e in log_lm if "accepted" in e)
    assert np.max(np.abs(T_gn - T_lm)) < 1e-6


@pytest.mark.parametrize("s", [0.95, 1.05])
def test_lm_sim3_recovers_depth_scale(s):
    sc = _box_world()
    cam = Camera(640, 480, 525.0, 525.0, 319.5, 239.5)
    T = synth.room_pose(40)
    live = render_frame(sc, cam, T, depth_scale=s)["depth"]
    dT0 = synth.perturb_pose(0.01, math.radians(1.0), np.random.default_rng(6))
    dT0[:3, :3] *= 1.015 / s
    dT, log = O.icp_lm(live, cam, _model_levels(sc, cam, T), dT0, dim=7, iters=(30, 15, 15))
    scale = np.cbrt(np.linalg.det(dT[:3, :3]))
    assert abs(scale - 1.0 / s) < 1e-6
    np.testing.assert_allclose(dT[:3, 3], 0, atol=1e-6)
    assert any(not e["accepted"] for e in log if "accepted" in e) or len(log) > 3


def test_anchoring_removes_a_common_drift():
    true = np.array([1.0, 1.05, 0.975, 1.025, 0.95])
    est = np.log(1.0 / true) + 0.013          # every estimate drifted by the same amount
    comp = O.anchored_log_scales(est, est[0])
    np.testing.assert_allclose(np.exp(comp), true[0] / true, rtol=1e-12)
