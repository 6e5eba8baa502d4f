"""Continuous batching of render + ICP requests from several sensors over one resident map.

A request carries a live depth frame of one sensor (any resolution, intrinsics and depth
scale), the pose to render the model at, and a prior offset.  Its work is a three-level model
render (one view per pyramid level) and coarse-to-fine point-to-plane ICP in Sim(3)
(or SE(3)) with the live frame, the scale factor of the sensor being part of the estimate.

The server runs in rounds.  At the start of a round every request whose arrival time has
passed is admitted while a slot is free and its buffers, sized for its own sensor, can be
carved out of the server's device arena (one allocation whose size is a budget taken from
the device's free memory at start-up); the
model pyramids of all newly admitted requests are rendered in one `dtsdf_render_batch`
launch, and every admitted request then advances by one ICP iteration in one
`icp_step_batch` (poses, convergence flags and results stay in device memory).  A request
leaves after its last iteration of the finest level; its slot and its part of the arena are
freed for the next round.  Requests that arrive while others are on the device therefore join the running
batch (continuous batching, not a queue in front of a serial worker), and each request's
result is bitwise the same as when it is served alone.

The iteration schedule is fixed (convergence only clears a device flag), so the host never
waits for a round: it enqueues rounds back to back and, for each request that leaves, a
copy of its pose into pinned memory followed by an event; the request is complete when the
host sees that event.
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import deque
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import dtsdf


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds from the start of the run
    sensor: int
    live_depth: torch.Tensor       # (H, W) float32 on the device
    T_model: np.ndarray            # camera-to-world pose the model is rendered at
    dT0: np.ndarray                # initial live -> model transform (4x4, may carry scale)
    # filled by the server
    admitted: float = math.nan
    finished: float = math.nan
    pose: Optional[np.ndarray] = None
    error: float = math.nan        # residual sum of squares of the last ICP step
    inliers: int = 0               # correspondences of the last ICP step
    H: Optional[np.ndarray] = None # normal matrix of the last ICP step (server only)
    slot: int = -1                 # slot that served it (server only)


@dataclasses.dataclass
class _Slot:
    pose: torch.Tensor
    active: torch.Tensor
    result: torch.Tensor
    live_levels: list = dataclasses.field(default_factory=list)   # per level depth, vertex, normal
    model_levels: list = dataclasses.field(default_factory=list)  # per level vertex, normal, mask
    req: Optional[Request] = None
    level: int = 0
    it: int = 0
    block: Optional[tuple] = None  # (offset, bytes) of the request's buffers in the arena
    c_req: object = None           # C descriptor of the current level's ICP request
    stage: Optional[torch.Tensor] = None   # pinned initial pose being copied in


_ALIGN = 256


def _buffers(cam, levels: int):
    """Buffers of one request, in arena order: per level the live depth, vertex and normal
    (float32: 1, 3, 3 per pixel) and the model vertex, normal (float32, 3 each) and mask
    (uint8, 1).  Returns [(level, side, name, dtype, elements)]."""
    out = []
    for l in range(levels):
        n = (cam.width >> l) * (cam.height >> l)
        out += [(l, "live", "depth", torch.float32, n),
                (l, "live", "vertex", torch.float32, 3 * n),
                (l, "live", "normal", torch.float32, 3 * n),
                (l, "model", "vertex", torch.float32, 3 * n),
                (l, "model", "normal", torch.float32, 3 * n),
                (l, "model", "mask", torch.uint8, n)]
    return out


def _aligned(nbytes: int) -> int:
    return (nbytes + _ALIGN - 1) // _ALIGN * _ALIGN


def _nbytes(dtype, count: int) -> int:
    return count * (4 if dtype == torch.float32 else 1)


def request_bytes(cam, levels: int = 3) -> int:
    """Device memory one request of this sensor holds while admitted: per level live depth,
    vertex and normal (28 B/px) and model vertex, normal and mask (25 B/px), each buffer
    starting on a 256-byte boundary of the arena."""
    return sum(_aligned(_nbytes(dt, k)) for _, _, _, dt, k in _buffers(cam, levels))


class Arena:
    """First-fit allocator over one device allocation of `nbytes` (offsets and sizes in
    multiples of 256 bytes; a freed range merges with its free neighbours).  All work on
    the memory is issued on one stream, so a range handed out again is only written after
    the earlier work on it."""

    def __init__(self, nbytes: int, device):
        self.size = nbytes // _ALIGN * _ALIGN
        self.mem = torch.empty(self.size, dtype=torch.uint8, device=device)
        self.free = [(0, self.size)] if self.size else []   # sorted, disjoint, not adjacent
        self.in_use = 0

    def alloc(self, nbytes: int) -> Optional[int]:
        nbytes = _aligned(nbytes)
        for i, (off, size) in enumerate(self.free):
            if size >= nbytes:
                if size == nbytes:
                    del self.free[i]
                else:
                    self.free[i] = (off + nbytes, size - nbytes)
                self.in_use += nbytes
                return off
        return None

    def release(self, off: int, nbytes: int) -> None:
        nbytes = _aligned(nbytes)
        self.in_use -= nbytes
        i = 0
        while i < len(self.free) and self.free[i][0] < off:
            i += 1
        self.free.insert(i, (off, nbytes))
        if i + 1 < len(self.free) and off + nbytes == self.free[i + 1][0]:
            self.free[i] = (off, nbytes + self.free[i + 1][1])
            del self.free[i + 1]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == off:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            del self.free[i]

    def view(self, off: int, dtype, count: int) -> torch.Tensor:
        return self.mem[off:off + _nbytes(dtype, count)].view(dtype)


class Server:
    def __init__(self, gmap: dtsdf.Map, sensors: Sequence, *, slots: int = 32,
                 budget_bytes: Optional[int] = None, memory_fraction: float = 0.01,
                 dim: int = 7, iters=(10, 5, 4),
                 params: dtsdf.IcpParams = dtsdf.IcpParams(), min_step: float = 1e-6,
                 z_near: float = 0.2, z_far: float = 10.0, stream=None):
        """`slots`: most requests on the device at once (the largest batch).  The request
        buffers come out of one device allocation of `budget_bytes`, or of
        `memory_fraction` of the device memory free at start-up (hipMemGetInfo); a request
        is admitted only when its own sensor's buffers fit in what is left of it."""
        self.map = gmap
        self.sensors = list(sensors)          # list of (cam, depth_scale)
        self.dim = dim
        self.iters = tuple(iters)
        self.L = len(self.iters)
        self.params = params
        self.min_step = min_step
        self.z_near, self.z_far = z_near, z_far
        self.stream = stream
        dev = torch.device("cuda", torch.cuda.current_device())
        free, _ = torch.cuda.mem_get_info(dev)
        biggest = max(request_bytes(c, self.L) for c, _ in self.sensors)
        self.budget = int(budget_bytes if budget_bytes is not None else memory_fraction * free)
        if self.budget < biggest:
            raise ValueError(f"memory budget {self.budget} B is below one request of the "
                             f"largest sensor ({biggest} B)")
        if self.budget > free:
            raise ValueError(f"memory budget {self.budget} B exceeds the free device memory "
                             f"({free} B)")
        if slots < 1:
            raise ValueError("at least one slot is needed")
        self.arena = Arena(self.budget, dev)
        self.peak_bytes = 0
        self._slots: List[_Slot] = [
            _Slot(pose=torch.zeros((4, 4), dtype=torch.float64, device=dev),
                  active=torch.zeros(1, dtype=torch.int32, device=dev),
                  result=torch.zeros(dtsdf.ICP_RESULT_BYTES, dtype=torch.uint8, device=dev))
            for _ in range(slots)]
        self.rounds = 0
        self.batch_sizes: List[int] = []
        self.deferred = 0      # rounds whose next admission waited for memory

    @property
    def in_use(self) -> int:
        return self.arena.in_use

    @property
    def slots_count(self) -> int:
        return len(self._slots)

    def _carve(self, s: _Slot, req: Request) -> bool:
        """Carves the request's buffers out of the arena into the slot; False if they do
        not fit."""
        cam, _ = self.sensors[req.sensor]
        need = request_bytes(cam, self.L)
        off = self.arena.alloc(need)
        if off is None:
            return False
        s.block = (off, need)
        s.live_levels = [dict() for _ in range(self.L)]
        s.model_levels = [dict() for _ in range(self.L)]
        o = off
        for l, side, name, dt, k in _buffers(cam, self.L):
            (s.live_levels if side == "live" else s.model_levels)[l][name] = \
                self.arena.view(o, dt, k)
            o += _aligned(_nbytes(dt, k))
        self.peak_bytes = max(self.peak_bytes, self.arena.in_use)
        return True

    # -- per-request set-up --------------------------------------------------------------
    def _views(self, s: _Slot, req: Request):
        cam, scale = self.sensors[req.sensor]
        views = []
        for l in range(self.L):
            c = dtsdf.level_camera(cam, l)
            n = c.width * c.height
            mb = s.model_levels[l]
            out = dict(vertex=mb["vertex"][:3 * n], normal=mb["normal"][:3 * n],
                       mask=mb["mask"][:n])
            views.append((c, req.T_model, self.z_near, self.z_far, out))
        return views

    def _prepare_live(self, s: _Slot, req: Request):
        cam, scale = self.sensors[req.sensor]
        d = req.live_depth.reshape(-1)
        for l in range(self.L):
            c = dtsdf.level_camera(cam, l)
            n = c.width * c.height
            lb = s.live_levels[l]
            if l == 0:
                lb["depth"][:n].copy_(d)
            else:
                p = dtsdf.level_camera(cam, l - 1)
                src = s.live_levels[l - 1]["depth"][:p.width * p.height].view(p.height, p.width)
                dtsdf._check(dtsdf._lib.dtsdf_depth_downsample(
                    dtsdf._dev_ptr(src, torch.float32), p.width, p.height,
                    dtsdf._dev_ptr(lb["depth"], torch.float32), dtsdf._stream(self.stream)),
                    "dtsdf_depth_downsample")
            dtsdf._check(dtsdf._lib.dtsdf_vertex_normal(
                dtsdf._dev_ptr(lb["depth"], torch.float32), dtsdf.ctypes.byref(dtsdf._intr(c)),
                1.0, dtsdf._dev_ptr(lb["vertex"], torch.float32),
                dtsdf._dev_ptr(lb["normal"], torch.float32), dtsdf._stream(self.stream)),
                "dtsdf_vertex_normal")

    def _icp_request(self, s: _Slot) -> dtsdf.IcpRequest:
        cam, _ = self.sensors[s.req.sensor]
        c = dtsdf.level_camera(cam, s.level)
        n = c.width * c.height
        lb, mb = s.live_levels[s.level], s.model_levels[s.level]
        return dtsdf.IcpRequest(lb["vertex"][:3 * n], lb["normal"][:3 * n], c,
                                mb["vertex"][:3 * n], mb["normal"][:3 * n], mb["mask"][:n], c,
                                s.pose, s.active, s.result, dim=self.dim, params=self.params,
                                min_step=self.min_step)

    # -- the loop --------------------------------------------------------------------------
    def run(self, requests: Sequence[Request], *, realtime: bool = True) -> List[Request]:
        """Serves `requests` (sorted by arrival).  With realtime, arrivals follow the wall
        clock from the start of the call; otherwise every request is available at once."""
        queue = deque(sorted(requests, key=lambda r: r.arrival))
        stream = self.stream if self.stream is not None else torch.cuda.current_stream()
        with torch.cuda.stream(stream):
            return self._run(queue, stream, realtime)

    def _run(self, queue, stream, realtime: bool) -> List[Request]:
        done: List[Request] = []
        leaving = []        # (event, request, pinned pose, pinned result)
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0   # noqa: E731
        while queue or leaving or any(s.req is not None for s in self._slots):
            # requests whose last round has completed on the device
            if leaving:
                still = []
                for item in leaving:
                    ev, req, hp, hr = item
                    if ev.query():
                        req.finished = now()
                        req.pose = hp.numpy().copy()
                        res = dtsdf.decode_result(hr, self.dim)
                        req.error, req.inliers, req.H = (float(res["error"]),
                                                         int(res["inliers"]), res["H"])
                        done.append(req)
                    else:
                        still.append(item)
                leaving = still
            # admission: arrived requests, free slot, memory budget
            new_views = []
            t = now()
            for si, s in enumerate(self._slots):
                if not queue or (realtime and queue[0].arrival > t):
                    break
                if s.req is not None:
                    continue
                if not self._carve(s, queue[0]):
                    self.deferred += 1
                    break
                req = queue.popleft()
                req.admitted = t
                req.slot = si
                s.req, s.level, s.it = req, self.L - 1, 0
                self._prepare_live(s, req)
                s.stage = torch.from_numpy(np.ascontiguousarray(req.dT0, np.float64)).pin_memory()
                s.pose.copy_(s.stage, non_blocking=True)
                s.active.fill_(1)
                new_views += self._views(s, req)
                s.c_req = dtsdf.icp_request_struct(self._icp_request(s))
            busy = [s for s in self._slots if s.req is not None]
            if not busy:
                if not leaving and queue and realtime:
                    time.sleep(max(0.0, min(queue[0].arrival - now(), 0.002)))
                continue
            if new_views:
                self.map.render_batch(new_views, stream=self.stream)
            dtsdf.icp_step_batch_structs([s.c_req for s in busy], stream=self.stream)
            self.batch_sizes.append(len(busy))
            self.rounds += 1
            for s in busy:
                s.it += 1
                if s.it < self.iters[s.level]:
                    continue
                s.level -= 1
                s.it = 0
                if s.level >= 0:
                    s.active.fill_(1)          # the next level starts afresh
                    s.c_req = dtsdf.icp_request_struct(self._icp_request(s))
                    continue
                # last round of this request: copy its pose and result out, then free the
                # slot (later work on the slot's buffers is ordered after these copies)
                hp = torch.empty((4, 4), dtype=torch.float64, pin_memory=True)
                hr = torch.empty(dtsdf.ICP_RESULT_BYTES, dtype=torch.uint8, pin_memory=True)
                hp.copy_(s.pose, non_blocking=True)
                hr.copy_(s.result, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(stream)
                leaving.append((ev, s.req, hp, hr))
                # the buffers stay readable through the slot until the memory is handed out
                # again (later work on it is ordered after this request's on the stream)
                self.arena.release(*s.block)
                s.block = None
                s.req = None
        return done


def serve_serial(gmap: dtsdf.Map, sensors: Sequence, requests: Sequence[Request], *, dim: int = 7,
                 iters=(10, 5, 4), params: dtsdf.IcpParams = dtsdf.IcpParams(),
                 min_step: float = 1e-6, z_near: float = 0.2, z_far: float = 10.0,
                 realtime: bool = True) -> List[Request]:
    """Baseline: one request at a time with the unbatched calls (three renders, per-level
    vertex/normal, icp_step with a host round-trip per iteration), in arrival order."""
    out = []
    t0 = time.perf_counter()
    for req in sorted(requests, key=lambda r: r.arrival):
        if realtime:
            wait = req.arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
        req.admitted = time.perf_counter() - t0
        cam, _ = sensors[req.sensor]
        levels = []
        for l in range(len(iters)):
            c = dtsdf.level_camera(cam, l)
            o = gmap.render(c, req.T_model, z_near, z_far, outputs=("vertex", "normal", "mask"))
            levels.append((o["vertex"], o["normal"], o["mask"], c))
        T, log = dtsdf.icp(req.live_depth, cam, levels, req.dT0, dim=dim, iters=iters,
                           params=params, min_step=min_step)
        req.finished = time.perf_counter() - t0
        req.pose = T
        if log:
            req.error, req.inliers = float(log[-1]["err"]), int(log[-1]["inliers"])
        out.append(req)
    return out


def latency_stats(reqs: Sequence[Request]) -> dict:
    lat = np.array([r.finished - r.arrival for r in reqs]) * 1e3
    return dict(p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                mean_ms=float(lat.mean()), max_ms=float(lat.max()))
