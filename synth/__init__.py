"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package generates inputs only: analytic scenes (spheres, boxes, thin plates, a closed
room), camera trajectories, depth and colour images obtained by intersecting camera rays with
those primitives, sensor noise and request streams.  It contains no part of the Directional
TSDF method itself (no fusion, no rendering of the map, no registration), so that the oracle
and the HIP path can both consume it without sharing any of the method's arithmetic.
"""
from .scenes import (  # noqa: F401
    Camera, Sphere, Box, Room, Scene, look_at, raycast_scene, render_frame,
    tiny_scene, tiny_cameras, tiny_frames, tiny_render_pose,
    room_scene, room_pose, room_frames, room_camera,
    tracking_cases, precision_scale, serving_sensors, serving_requests, serving_workload,
    perturb_pose, random_rotation_small,
)
