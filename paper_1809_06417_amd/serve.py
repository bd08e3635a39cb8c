"""Serving loop for per-frame reconstruction jobs with continuous batching.

Jobs (one video frame each: frames, the frame's extinction, a fixed number of
SART iterations, warm-started from the video's previous result) arrive over
time. The loop admits waiting jobs whenever their video is idle, a batch slot
is free and the video's plan fits in the HBM budget (idle plans are evicted,
least recently used first; every video's latest volume stays resident on the
device). All admitted jobs then advance together, one iteration per step,
each step being one batched launch per phase (rte_job_step); a job leaves the
batch when its iterations are done and the next one can join at the very next
step. Per-job results are bitwise the ones each job gets alone.

The one-job-at-a-time reference (`serve_sequential`) runs the same jobs in
arrival order with rte_reconstruct.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import rte

__all__ = ["Job", "VideoState", "serve", "serve_sequential", "latency_summary"]


@dataclasses.dataclass
class Job:
    jid: int
    video: int
    frame: int
    arrival: float                      # seconds after the start of the run
    frames: object = None               # device tensor [V, C, H, W]
    extinction: object = None           # device tensor [nz, ny, nx]
    start: float | None = None
    done: float | None = None
    iters: int = 0
    result: object = None               # copy of the result (keep_results)


class VideoState:
    def __init__(self, spec, channels=3):
        self.spec = spec
        self.channels = channels
        self.plan = None
        self.plan_bytes = rte.workspace_bytes(spec.grid, spec.rig, channels=channels)
        self.volume = None       # latest result, resident on the device
        self.resident = False    # the plan's packed volume holds self.volume
        self.busy = False
        self.last_used = -1.0

    def ensure_plan(self):
        if self.plan is None:
            self.plan = rte.Plan(self.spec.grid, self.spec.rig, channels=self.channels)
            self.resident = False
        return self.plan

    def evict(self):
        if self.plan is not None:
            self.plan.close()
            self.plan = None
            self.resident = False


def latency_summary(jobs):
    lat = np.array([j.done - j.arrival for j in jobs])
    span = max(j.done for j in jobs) - min(j.arrival for j in jobs)
    return {"jobs": len(jobs), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "frames_per_s": len(jobs) / span, "span_s": span}


def _zeros_volume(vs):
    import torch
    g = vs.spec.grid
    return torch.zeros((vs.channels,) + g.shape_zyx, device="cuda")


def serve(videos, jobs, iters=10, hbm_budget_bytes=32 << 30, max_batch=64, keep_results=False,
          clock=time.perf_counter, log=None):
    """Run `jobs` (sorted by arrival) through the continuous-batching loop.
    videos: {video id: VideoState}. Returns the jobs with start/done times."""
    import torch
    for j in jobs:
        if videos[j.video].plan_bytes > hbm_budget_bytes:
            raise ValueError(f"video {j.video} needs {videos[j.video].plan_bytes} B of workspace, "
                             f"more than the budget of {hbm_budget_bytes} B")
    pending = collections.deque(sorted(jobs, key=lambda j: j.arrival))
    waiting, active = [], []
    used = sum(v.plan.device_bytes for v in videos.values() if v.plan is not None)
    t0 = clock()
    steps = 0
    while pending or waiting or active:
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            waiting.append(pending.popleft())
        # admission: FIFO among jobs whose video is idle
        for job in list(waiting):
            if len(active) >= max_batch:
                break
            vs = videos[job.video]
            if vs.busy:
                continue
            if vs.plan is None:
                while used + vs.plan_bytes > hbm_budget_bytes:
                    idle = [v for v in videos.values() if v.plan is not None and not v.busy and v is not vs]
                    if not idle:
                        break
                    lru = min(idle, key=lambda v: v.last_used)
                    used -= lru.plan.device_bytes
                    lru.evict()
                if used + vs.plan_bytes > hbm_budget_bytes:
                    continue
                vs.ensure_plan()
                used += vs.plan.device_bytes
            warm = None if vs.resident else (vs.volume if vs.volume is not None else _zeros_volume(vs))
            vs.plan.job_begin(job.frames, job.extinction, warm)
            vs.busy = True
            job.start = clock() - t0
            job.iters = 0
            active.append(job)
            waiting.remove(job)
        if not active:
            if pending:
                time.sleep(max(0.0, min(pending[0].arrival - (clock() - t0), 0.05)))
            continue
        rte.job_step([videos[j.video].plan for j in active])
        steps += 1
        finished = []
        for j in active:
            j.iters += 1
            if j.iters == iters:
                vs = videos[j.video]
                if vs.volume is None:
                    vs.volume = _zeros_volume(vs)
                vs.plan.job_end(vs.volume)
                vs.resident = True
                if keep_results:
                    j.result = vs.volume.clone()
                finished.append(j)
        torch.cuda.synchronize()
        if finished:
            t = clock() - t0
            for j in finished:
                j.done = t
                vs = videos[j.video]
                vs.busy = False
                vs.last_used = t
                active.remove(j)
            if log:
                log(f"t={t:7.3f}s done {len(finished)} (active {len(active)}, waiting {len(waiting)})")
    return jobs


def serve_sequential(videos, jobs, iters=10, keep_results=False, clock=time.perf_counter):
    """Reference: one job at a time in arrival order (rte_reconstruct), same
    warm starts; all plans stay resident."""
    import torch
    order = sorted(jobs, key=lambda j: j.arrival)
    t0 = clock()
    for job in order:
        now = clock() - t0
        if job.arrival > now:
            time.sleep(job.arrival - now)
        vs = videos[job.video]
        plan = vs.ensure_plan()
        if vs.volume is None:
            vs.volume = _zeros_volume(vs)
        job.start = clock() - t0
        plan.reconstruct(job.frames, job.extinction, vs.volume, iters)
        if keep_results:
            job.result = vs.volume.clone()
        torch.cuda.synchronize()
        job.done = clock() - t0
    return jobs
