"""Continuous-batching render server over one resident Gaussian scene.

Requests (an ERP camera pose and resolution) arrive over time.  The server
keeps `slots` batches in flight, each on its own HIP stream (default
priority).  Whenever a slot is free, it forms a batch from the requests that
have arrived (FIFO, at most `max_batch`, at most `max_tiles` 16x16 tiles in
all -- larger batches of big images were measured slower than rendering
them one by one -- and only
while the estimated HBM footprint of everything in flight stays within
`hbm_budget`), and enqueues it
with one omnigs_forward_batch call in capacity mode: the instance buffers are
sized from a running per-resolution estimate, so the call never waits on the
device and the scheduler goes straight back to admitting and polling.
Completion is observed with a HIP event per batch; a batch whose instance
count overflowed its capacity is re-queued at the head of the queue with a
larger estimate (its outputs are discarded).

Each result equals the render of that request alone (the batched path is
bit-identical to omnigs_forward per camera), whatever it was batched with.

The one-request-at-a-time baseline is the same server with slots=1 and
max_batch=1: FIFO, one render at a time on one stream.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np
import torch

from . import omnigs as B

@dataclasses.dataclass
class Request:
    rid: int
    camera: dict          # R, t, width, height
    arrival: float        # seconds after the start of the run
    start: float = -1.0   # when its (last) batch was enqueued
    done: float = -1.0    # when its completion was observed
    batch_size: int = 0
    retries: int = 0
    image: torch.Tensor | None = None

    @property
    def latency(self):
        return self.done - self.arrival

    @property
    def pixels(self):
        return int(self.camera["width"]) * int(self.camera["height"])


def _tiles(camera) -> int:
    return ((int(camera["width"]) + 15) // 16) * ((int(camera["height"]) + 15) // 16)


def footprint(n_gaussians: int, cameras: list, instances: int) -> int:
    """HBM bytes of one batch: what omnigs_forward_batch allocates for these
    cameras and instance capacity (the library's own size query) plus the
    outputs the server allocates."""
    return (B.omnigs_forward_batch_bytes(n_gaussians, cameras, instances)
            + sum(B.output_bytes(c) for c in cameras))


class _Slot:
    def __init__(self, device):
        self.stream = torch.cuda.Stream(device)  # default priority
        self.event = torch.cuda.Event()
        self.flag = torch.empty(1, dtype=torch.int32, pin_memory=True)
        self.batch = None      # list of Request in flight
        self.result = None
        self.bytes = 0


class Server:
    """Continuous-batching server.  `instance_estimate` maps (width, height)
    to an instance count used to size capacities (learned upwards on
    overflow); `margin` scales it.  `keep_images`: True, False, or a set of
    request ids whose images are kept."""

    def __init__(self, gaussians: dict, settings: dict | None = None, slots: int = 2, max_batch: int = 8,
                 hbm_budget: int = 16 << 30, instance_estimate: dict | None = None, margin: float = 1.25,
                 keep_images=True, max_tiles: int = 1 << 16):
        if not 1 <= max_batch <= B.OMNIGS_MAX_BATCH:
            raise ValueError(f"max_batch must be in [1, {B.OMNIGS_MAX_BATCH}]")
        self.g = gaussians
        self.settings = settings
        self.device = gaussians["means"].device
        self.n = int(gaussians["means"].shape[0])
        self.slots = [_Slot(self.device) for _ in range(slots)]
        self.max_batch = max_batch
        self.budget = hbm_budget
        self.est = dict(instance_estimate or {})
        self.margin = margin
        self.keep_images = keep_images
        self.max_tiles = max_tiles
        self.overflows = 0
        self.batches = 0

    # ------------------------------------------------------------ sizing
    def instances_for(self, req: Request) -> int:
        key = (int(req.camera["width"]), int(req.camera["height"]))
        if key not in self.est:
            # scale the nearest known resolution by pixel count, else a
            # generous default of 16 instances per Gaussian
            if self.est:
                k2 = min(self.est, key=lambda k: abs(k[0] * k[1] - key[0] * key[1]))
                self.est[key] = int(self.est[k2] * max(1.0, key[0] * key[1] / (k2[0] * k2[1])))
            else:
                self.est[key] = 16 * self.n
        return int(self.est[key] * self.margin) + 1024

    def batch_bytes(self, batch: list) -> int:
        """Footprint of a batch with the capacity it is launched with."""
        cap = min(sum(self.instances_for(r) for r in batch), (1 << 32) - 1)
        return footprint(self.n, [r.camera for r in batch], cap)

    def calibrate(self, cameras):
        """Render each distinct resolution once alone (instance count read
        back) to seed the estimates."""
        for cam in cameras:
            key = (int(cam["width"]), int(cam["height"]))
            r = B.omnigs_forward_batch(self.g, [cam], self.settings, instance_capacity=0)
            self.est[key] = max(self.est.get(key, 0), r.n_instances)
        torch.cuda.synchronize(self.device)

    # ---------------------------------------------------------- launching
    def _launch(self, slot: _Slot, batch: list, now: float):
        cap = sum(self.instances_for(r) for r in batch)
        cap = min(cap, (1 << 32) - 1)
        with torch.cuda.stream(slot.stream):
            res = B.omnigs_forward_batch(self.g, [r.camera for r in batch], self.settings, instance_capacity=cap)
            slot.flag.copy_(res.overflow, non_blocking=True)
            slot.event.record(slot.stream)
        for r in batch:
            r.start = now
            r.batch_size = len(batch)
        slot.batch, slot.result = batch, res
        slot.bytes = self.batch_bytes(batch)
        self.batches += 1

    def _finish(self, slot: _Slot, now: float, queue: collections.deque, done: list):
        batch, res = slot.batch, slot.result
        slot.batch = slot.result = None
        slot.bytes = 0
        if int(slot.flag[0]) != 0:
            # capacity too small: grow the estimates and retry at the head
            self.overflows += 1
            for r in batch:
                key = (int(r.camera["width"]), int(r.camera["height"]))
                self.est[key] = 2 * self.est[key] + 1
                r.retries += 1
            for r in reversed(batch):
                queue.appendleft(r)
            return
        for r, o in zip(batch, res.outs):
            r.done = now
            keep = self.keep_images is True or (self.keep_images and r.rid in self.keep_images)
            r.image = o["image"] if keep else None
            done.append(r)

    def run(self, requests: list, clock=time.perf_counter, idle_sleep: float = 0.0) -> dict:
        """Serve `requests` (arrival times relative to the start).  Returns
        the summary; each Request gets start / done / image."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue = collections.deque()
        done = []
        t0 = clock()
        while pending or queue or any(s.batch is not None for s in self.slots):
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            for s in self.slots:
                if s.batch is not None and s.event.query():
                    self._finish(s, clock() - t0, queue, done)
            in_flight = sum(s.bytes for s in self.slots)
            for s in self.slots:
                if s.batch is not None or not queue:
                    continue
                # admit while the footprint fits; a request larger than the
                # whole budget still runs, alone, when nothing else is in flight
                batch, need, tiles = [], 0, 0
                while queue and len(batch) < self.max_batch:
                    b = self.batch_bytes(batch + [queue[0]])
                    if in_flight + b > self.budget and (batch or in_flight > 0):
                        break
                    t = _tiles(queue[0].camera)
                    if batch and tiles + t > self.max_tiles:
                        break
                    batch.append(queue.popleft())
                    need = b
                    tiles += t
                if not batch:
                    break
                self._launch(s, batch, clock() - t0)
                in_flight += need
            if idle_sleep and not queue and pending:
                time.sleep(min(idle_sleep, max(0.0, pending[0].arrival - (clock() - t0))))
        makespan = max(r.done for r in done) - min(r.arrival for r in done) if done else 0.0
        lat = np.array([r.latency for r in done]) * 1e3
        return dict(requests=len(done), renders_per_s=len(done) / makespan if makespan > 0 else 0.0,
                    p50_ms=float(np.percentile(lat, 50)) if len(lat) else None,
                    p99_ms=float(np.percentile(lat, 99)) if len(lat) else None,
                    mean_batch=float(np.mean([r.batch_size for r in done])) if done else 0.0,
                    batches=self.batches, overflows=self.overflows, makespan_s=makespan)


SCENE_KEYS = ("means", "scales", "quats", "opacities", "sh")


def save_scene(path: str, g: dict) -> None:
    """Write a resident scene (activated parameters, as omnigs_forward takes
    them) to an .npz file: float32 arrays and the SH degree, nothing pickled."""
    arrays = {k: (g[k].detach().cpu().numpy() if isinstance(g[k], torch.Tensor) else np.asarray(g[k]))
              .astype(np.float32) for k in SCENE_KEYS}
    np.savez(path, sh_degree=np.int32(g["sh_degree"]), **arrays)


def load_scene(path: str, device) -> dict:
    """Read a scene written by save_scene onto `device` (contiguous float32
    tensors), checking the array shapes against each other."""
    with np.load(path, allow_pickle=False) as f:
        g = {k: torch.from_numpy(np.ascontiguousarray(f[k], dtype=np.float32)).to(device) for k in SCENE_KEYS}
        g["sh_degree"] = int(f["sh_degree"])
    n = g["means"].shape[0]
    shapes = dict(means=(n, 3), scales=(n, 3), quats=(n, 4), opacities=(n,))
    for k, shp in shapes.items():
        if tuple(g[k].shape) != shp:
            raise ValueError(f"{path}: {k} has shape {tuple(g[k].shape)}, expected {shp}")
    if g["sh"].dim() != 3 or g["sh"].shape[0] != n or g["sh"].shape[2] != 3 or \
            not (g["sh_degree"] + 1) ** 2 <= g["sh"].shape[1] <= 16:
        raise ValueError(f"{path}: sh has shape {tuple(g['sh'].shape)} for degree {g['sh_degree']}")
    return g


def make_requests(cameras: list, arrivals=None) -> list:
    """Requests for `cameras` in order, arriving at `arrivals` (seconds; None:
    all at 0)."""
    return [Request(k, cam, float(arrivals[k]) if arrivals is not None else 0.0) for k, cam in enumerate(cameras)]
