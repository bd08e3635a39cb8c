"""Serving loop for per-frame reconstruction jobs with continuous batching.

Jobs (one video frame each: frames, the frame's extinction, a fixed number of
SART iterations, warm-started from the video's previous result) arrive over
time. The loop admits waiting jobs whenever their video is idle, a batch slot
is free, the device memory the job needs fits the HBM budget, and either
nothing runs or a backlog has formed (at least `share_backlog` jobs wait;
without one, sharing the GPU would lengthen the running jobs about as much as
waiting lengthens the new one, so a lone arrival waits its turn): the video's
plan workspace, its resident volume and the job's frames and extinction
(idle plans are evicted, least recently used first; every video's latest
volume stays resident on the device to warm-start its next frame).

Admitted jobs are spread over `lanes` HIP streams (the lane with the fewest
march samples per iteration takes the next job, for the job's whole life).
Each lane advances all of its jobs together, one iteration per batched
launch per phase (rte_job_step), and keeps up to `depth` steps queued ahead
of the GPU, so one lane's render runs beside another lane's back-projection
and the GPU never waits for the host between steps. A job leaves its lane
when its iterations are enqueued; a completion event recorded after its last
kernels tells the host when it is done (no device-wide synchronisation), and
the next job of the same video is admitted only then. Every job runs the same
kernels in the same order on one stream, so its result is bitwise the one it
gets alone.

The one-job-at-a-time reference (`serve_sequential`) runs the same jobs in
arrival order with rte_reconstruct on one stream.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import rte

__all__ = ["Job", "VideoState", "serve", "serve_sequential", "latency_summary", "min_budget"]


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
    lane: int = -1

    def input_bytes(self):
        return 4 * (self.frames.numel() + self.extinction.numel())


class VideoState:
    def __init__(self, spec, channels=3):
        self.spec = spec
        self.channels = channels
        self.plan = None
        self.plan_bytes = rte.workspace_bytes(spec.grid, spec.rig, channels=channels)
        g = spec.grid
        self.volume_bytes = 4 * channels * g.nx * g.ny * g.nz
        self.samples = None      # march samples per iteration (known once a plan exists)
        self.volume = None       # latest result, resident on the device
        self.resident = False    # the plan's packed volume holds self.volume
        self.busy = False
        self.last_used = -1.0

    def ensure_plan(self):
        if self.plan is None:
            self.plan = rte.Plan(self.spec.grid, self.spec.rig, channels=self.channels)
            self.samples = self.plan.samples
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


def min_budget(videos, jobs):
    """Smallest HBM budget that admits every job: the largest plan, every
    video's resident volume and the largest job's inputs."""
    return (max(v.plan_bytes for v in videos.values()) + sum(v.volume_bytes for v in videos.values())
            + max(j.input_bytes() for j in jobs))


def _zeros_volume(vs):
    import torch
    g = vs.spec.grid
    return torch.zeros((vs.channels,) + g.shape_zyx, device="cuda")


def serve(videos, jobs, iters=10, hbm_budget_bytes=32 << 30, max_batch=64, keep_results=False,
          clock=time.perf_counter, log=None, lanes=2, depth=2, stats=None, share_backlog=3):
    """Run `jobs` (sorted by arrival) through the continuous-batching loop.
    videos: {video id: VideoState}. Returns the jobs with start/done times.
    stats (a dict, optional) receives the GPU-busy fraction of the span (time
    with at least one step or job end not yet complete) and the step count.
    share_backlog: a waiting job joins running ones only while at least this
    many jobs wait (None: whenever it can)."""
    import torch
    need = min_budget(videos, jobs) if jobs else 0
    if need > hbm_budget_bytes:
        raise ValueError(f"the jobs need at least {need} B (largest plan, resident volumes, largest job "
                         f"inputs), more than the budget of {hbm_budget_bytes} B")
    streams = [torch.cuda.Stream() for _ in range(lanes)]  # default priority
    pending = collections.deque(sorted(jobs, key=lambda j: j.arrival))
    waiting = []
    lane_jobs = [[] for _ in range(lanes)]
    inflight = [collections.deque() for _ in range(lanes)]   # events after each queued step
    finishing = []                                           # (job, event after its job end)

    def used_bytes():
        n = sum(v.plan.device_bytes for v in videos.values() if v.plan is not None)
        n += sum(v.volume_bytes for v in videos.values() if v.volume is not None)
        n += sum(j.input_bytes() for lj in lane_jobs for j in lj)
        n += sum(j.input_bytes() for j, _ in finishing)
        return n

    t0 = clock()
    steps = 0
    busy_s = 0.0
    t_prev = 0.0
    while pending or waiting or finishing or any(lane_jobs):
        now = clock() - t0
        if any(inflight) or finishing:
            busy_s += now - t_prev
        t_prev = now
        while pending and pending[0].arrival <= now:
            waiting.append(pending.popleft())
        # completions
        for l in range(lanes):
            while inflight[l] and inflight[l][0].query():
                inflight[l].popleft()
        for item in list(finishing):
            job, ev = item
            if ev.query():
                t = clock() - t0
                job.done = t
                vs = videos[job.video]
                vs.busy = False
                vs.last_used = t
                finishing.remove(item)
                if log:
                    log(f"t={t:7.3f}s done job {job.jid} (waiting {len(waiting)})")
        # admission: FIFO among jobs whose video is idle
        n_active = sum(len(lj) for lj in lane_jobs)
        for job in list(waiting):
            if n_active >= max_batch:
                break
            if share_backlog is not None and n_active > 0 and len(waiting) < share_backlog:
                break
            vs = videos[job.video]
            if vs.busy:
                continue
            extra = job.input_bytes() + (vs.volume_bytes if vs.volume is None else 0)
            if vs.plan is None:
                extra += vs.plan_bytes
                while used_bytes() + extra > hbm_budget_bytes:
                    idle = [v for v in videos.values() if v.plan is not None and not v.busy and v is not vs]
                    if not idle:
                        break
                    min(idle, key=lambda v: v.last_used).evict()
            if used_bytes() + extra > hbm_budget_bytes:
                continue
            vs.ensure_plan()
            lane = min(range(lanes), key=lambda l: sum(videos[j.video].samples for j in lane_jobs[l]))
            with torch.cuda.stream(streams[lane]):
                if vs.volume is None:
                    vs.volume = _zeros_volume(vs)
                warm = None if vs.resident else vs.volume
                vs.plan.job_begin(job.frames, job.extinction, warm)
            vs.busy = True
            job.start = clock() - t0
            job.iters = 0
            job.lane = lane
            lane_jobs[lane].append(job)
            waiting.remove(job)
            n_active += 1
        # issue: each lane keeps up to `depth` steps queued
        issued = False
        for l in range(lanes):
            if not lane_jobs[l] or len(inflight[l]) >= depth:
                continue
            with torch.cuda.stream(streams[l]):
                rte.job_step([videos[j.video].plan for j in lane_jobs[l]])
                steps += 1
                for j in list(lane_jobs[l]):
                    j.iters += 1
                    if j.iters == iters:
                        vs = videos[j.video]
                        vs.plan.job_end(vs.volume)
                        vs.resident = True
                        if keep_results:
                            j.result = vs.volume.clone()
                        ev = torch.cuda.Event()
                        ev.record(streams[l])
                        finishing.append((j, ev))
                        lane_jobs[l].remove(j)
                ev = torch.cuda.Event()
                ev.record(streams[l])
                inflight[l].append(ev)
            issued = True
        if not issued:
            # nothing to enqueue: wait a little for a completion or an arrival
            time.sleep(0.0002 if (any(inflight) or finishing) else
                       max(0.0, min(pending[0].arrival - (clock() - t0), 0.05)) if pending else 0.0002)
    for st in streams:
        st.synchronize()
    if stats is not None:
        span = max(j.done for j in jobs) - min(j.arrival for j in jobs) if jobs else 0.0
        stats.update({"gpu_busy": busy_s / span if span > 0 else 0.0, "steps": steps, "lanes": lanes,
                      "depth": depth})
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
