"""Serving: the job API (rte_job_begin / rte_job_step / rte_job_end) and the
continuous-batching loop. Batched steps must give every job bitwise the result
it gets alone, the job path must equal rte_reconstruct, and at a small size
both agree with the FP64 oracle's reconstruction."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from gpu_util import VOLUME_RMS, as64, dev, f32, host, rel_rms, say

pytestmark = pytest.mark.gpu


def rte():
    from paper_1809_06417_amd import rte as _rte
    return _rte


def small_spec(video, n, views, W, H):
    """A seeded video spec with its grid and rig shrunk to oracle-friendly sizes."""
    spec = synth.video_spec(video, seed=5)
    return dataclasses.replace(spec, grid=synth.Grid(n, n, n),
                               rig=synth.ring_rig(views, W, H, elevation_jitter_deg=10.0, seed=50 + video))


SMALL = [small_spec(0, 20, 3, 40, 32), small_spec(1, 24, 4, 36, 36), small_spec(2, 17, 2, 48, 30)]


def frame_inputs(spec, frame):
    """(frames, extinction) of one frame; frames are FP64 oracle renders of the
    ground truth at that frame, rounded to FP32."""
    em, sig = synth.video_frame(spec, frame)
    em, sig = f32(em), f32(sig)
    F = oracle.render(spec.grid, spec.rig, as64(em), as64(sig), step_vox=0.5)
    return f32(F), sig


def new_plan(spec):
    return rte().Plan(spec.grid, spec.rig, channels=3, step_vox=0.5)


@pytest.mark.parametrize("update", ["sart", "mlem", "paper"])
def test_job_path_equals_reconstruct(update):
    import torch
    spec = SMALL[0]
    F, sig = frame_inputs(spec, 0)
    say("job vs reconstruct", update)
    with new_plan(spec) as p:
        start = dev(np.full((3,) + spec.grid.shape_zyx, 0.05))
        a = start.clone()
        p.reconstruct(dev(F), dev(sig), a, 4, update=update)
        b = torch.empty_like(start)
        p.job_begin(dev(F), dev(sig), start, update=update)
        for _ in range(4):
            rte().job_step([p])
        p.job_end(b)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        assert p.stats()[0] == 4


@pytest.mark.parametrize("update,restrict", [("sart", "mask"), ("mlem", "hull"), ("paper", "hull")])
def test_job_path_equals_reconstruct_with_restrictions(update, restrict):
    """Flame mask and visual hull: a job (its first step run alone, the
    rest batched with a second job) gives bitwise the rte_reconstruct result."""
    import torch
    spec, other = SMALL[1], SMALL[0]
    F, sig = frame_inputs(spec, 1)
    thr = float(np.float32(0.05 * F.max()))
    kw = dict(update=update, flame_threshold=thr, hull=restrict == "hull", outside_value=0.0)
    say("job vs reconstruct with", update, restrict)
    with new_plan(spec) as p, new_plan(other) as q:
        start = dev(np.full((3,) + spec.grid.shape_zyx, 0.05))
        a = start.clone()
        p.reconstruct(dev(F), dev(sig), a, 4, **kw)
        Fq, sq = frame_inputs(other, 0)
        q.job_begin(dev(Fq), dev(sq), torch.zeros((3,) + q.vol_shape, device="cuda"), update=update)
        rte().job_step([q])
        p.job_begin(dev(F), dev(sig), start, **kw)
        for _ in range(4):
            rte().job_step([q, p])   # p's first step runs alone, the later ones batched with q
        b = torch.empty_like(start)
        p.job_end(b)
        q.job_end(None)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        assert p.stats()[0] == 4


def test_batched_steps_match_each_job_alone():
    """Three plans of different grids, view counts and image sizes advance
    together; each result is bitwise its result alone."""
    import torch
    say("batched vs alone")
    plans = [new_plan(s) for s in SMALL]
    try:
        inputs = [frame_inputs(s, 3) for s in SMALL]
        alone = []
        for p, (F, sig) in zip(plans, inputs):
            out = torch.zeros((3,) + p.vol_shape, device="cuda")
            p.reconstruct(dev(F), dev(sig), out, 5)
            alone.append(out)
        held = [(dev(F), dev(sig)) for F, sig in inputs]
        for p, (Fd, sd) in zip(plans, held):
            p.job_begin(Fd, sd, torch.zeros((3,) + p.vol_shape, device="cuda"))
        # a ragged mix, five steps per plan: plan 2 joins one step late and
        # leaves one step late, and the first plan of a step varies
        for group in ([0, 1], [0, 1, 2], [1, 2], [2, 0], [0, 1, 2], [1, 0], [2]):
            rte().job_step([plans[i] for i in group])
        mixed = []
        for p in plans:
            out = torch.empty((3,) + p.vol_shape, device="cuda")
            p.job_end(out)
            mixed.append(out)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(alone, mixed)):
            assert torch.equal(a, b), i
    finally:
        for p in plans:
            p.close()


def test_warm_start_keeps_the_resident_volume():
    import torch
    spec = SMALL[1]
    (F0, s0), (F1, s1) = frame_inputs(spec, 0), frame_inputs(spec, 1)
    say("warm start")
    with new_plan(spec) as p:
        ref = torch.zeros((3,) + p.vol_shape, device="cuda")
        p.reconstruct(dev(F0), dev(s0), ref, 3)
        p.reconstruct(dev(F1), dev(s1), ref, 3)
        f0, f1 = dev(F0), dev(F1)
        p.job_begin(f0, dev(s0), torch.zeros_like(ref))
        for _ in range(3):
            rte().job_step([p])
        p.job_end(None)
        p.job_begin(f1, dev(s1), None)  # start from the resident result
        for _ in range(3):
            rte().job_step([p])
        out = torch.empty_like(ref)
        p.job_end(out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


def test_job_path_matches_oracle():
    spec = SMALL[2]
    F, sig = frame_inputs(spec, 2)
    em0 = np.zeros((3,) + spec.grid.shape_zyx)
    ref = oracle.reconstruct(spec.grid, spec.rig, as64(F), as64(sig), em0, 6)
    say("job vs oracle")
    import torch
    with new_plan(spec) as p:
        out = torch.empty((3,) + p.vol_shape, device="cuda")
        p.job_begin(dev(F), dev(sig), dev(em0))
        for _ in range(6):
            rte().job_step([p])
        p.job_end(out)
        got = host(out)
    assert rel_rms(got, ref) <= VOLUME_RMS


def test_job_api_rejects_bad_batches():
    import torch
    say("job errors")
    a, b = new_plan(SMALL[0]), rte().Plan(SMALL[1].grid, SMALL[1].rig, channels=1)
    try:
        F, sig = frame_inputs(SMALL[0], 0)
        with pytest.raises(rte().RteError):
            rte().job_step([a])                       # no open job
        with pytest.raises(rte().RteError):
            a.job_begin(dev(F), dev(sig), None, subsets=2)  # ordered subsets: not in jobs
        Fd = dev(F)
        a.job_begin(Fd, dev(sig), torch.zeros((3,) + a.vol_shape, device="cuda"))
        with pytest.raises(rte().RteError):
            a.job_begin(Fd, dev(sig), None)           # already open
        with pytest.raises(rte().RteError):
            rte().job_step([a, a])                    # listed twice
        F1 = torch.zeros((SMALL[1].rig.n_views, 1, SMALL[1].rig.height, SMALL[1].rig.width), device="cuda")
        b.job_begin(F1, torch.zeros(b.vol_shape, device="cuda"), torch.zeros((1,) + b.vol_shape, device="cuda"))
        with pytest.raises(rte().RteError):
            rte().job_step([a, b])                    # mixed channel counts
        before = torch.zeros((3,) + a.vol_shape, device="cuda")
        a.job_end(before)
        b.job_end(None)
        torch.cuda.synchronize()
        assert a.stats()[0] == 0                      # the rejected steps advanced nothing
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("budget, lanes, share", [("ample", 2, 3), ("one_plan", 2, 3), ("ample", 1, 3),
                                                   ("ample", 3, 3), ("ample", 2, None), ("one_plan", 2, None)])
def test_serving_loop_matches_sequential(budget, lanes, share):
    """The continuous-batching loop (on 1-3 stream lanes with steps queued
    ahead, with LRU eviction of idle plans when the HBM budget holds only
    one plan besides the resident volumes, sharing the GPU once three jobs
    wait or whenever a job can be admitted) returns, per job, bitwise the
    volume of the one-job-at-a-time reference in arrival order."""
    import torch
    from paper_1809_06417_amd import serve
    arrivals = synth.poisson_arrivals(12, 400.0, seed=2)
    vids = np.random.default_rng(4).integers(0, len(SMALL), size=len(arrivals))
    say("serving loop", budget, lanes, share)

    def make_jobs():
        count = {}
        jobs = []
        for i, (t, v) in enumerate(zip(arrivals, vids)):
            fr = count.get(int(v), 0)
            count[int(v)] = fr + 1
            F, sig = inputs[(int(v), fr)]
            jobs.append(serve.Job(i, int(v), fr, float(t), dev(F), dev(sig)))
        return jobs

    count = {}
    inputs = {}
    for v in vids:
        fr = count.get(int(v), 0)
        count[int(v)] = fr + 1
        inputs[(int(v), fr)] = frame_inputs(SMALL[int(v)], fr)

    videos = {i: serve.VideoState(s) for i, s in enumerate(SMALL)}
    cap = serve.min_budget(videos, make_jobs()) if budget == "one_plan" else 1 << 34
    st = {}
    jobs = serve.serve(videos, make_jobs(), iters=4, hbm_budget_bytes=cap, keep_results=True, lanes=lanes,
                       stats=st, share_backlog=share)
    assert 0.0 < st["gpu_busy"] <= 1.01
    for v in videos.values():
        v.evict()
    ref_videos = {i: serve.VideoState(s) for i, s in enumerate(SMALL)}
    ref = serve.serve_sequential(ref_videos, make_jobs(), iters=4, keep_results=True)
    for v in ref_videos.values():
        v.evict()
    torch.cuda.synchronize()
    for a, b in zip(sorted(jobs, key=lambda j: j.jid), sorted(ref, key=lambda j: j.jid)):
        assert a.done is not None and a.done >= a.arrival
        assert torch.equal(a.result, b.result), a.jid
    s = serve.latency_summary(jobs)
    assert s["jobs"] == 12 and s["p99_ms"] >= s["p50_ms"] > 0


def test_batched_inscatter_steps_match_each_job_alone():
    """Jobs with in-scattering: a step computes every plan's in-scatter grid
    with one launch per march pass and reduce. A volume beyond one slab (the
    slab-per-XCD schedule, five passes), two small one-pass volumes with
    other grid resolutions and direction counts, and a Henyey-Greenstein plan
    (per-view grids) advance in ragged groups; each result is bitwise its
    result alone (rte_reconstruct, per-plan launches)."""
    import torch
    say("batched in-scatter vs alone")
    cfgs = [dict(n=96, views=3, W=40, H=36, M=12, dirs=16, g=0.0),
            dict(n=24, views=4, W=36, H=36, M=8, dirs=12, g=0.0),
            dict(n=20, views=2, W=32, H=30, M=6, dirs=9, g=0.0),
            dict(n=22, views=3, W=30, H=28, M=7, dirs=10, g=0.5)]
    plans, inputs = [], []
    try:
        for i, c in enumerate(cfgs):
            spec = small_spec(i, c["n"], c["views"], c["W"], c["H"])
            plans.append(rte().Plan(spec.grid, spec.rig, channels=3, step_vox=0.5, albedo=0.3,
                                    scatter_res=c["M"], scatter_dirs=c["dirs"], phase_g=c["g"]))
            em, sig = synth.video_frame(spec, 2)
            emd, sgd = dev(em), dev(sig)
            S = plans[-1].inscatter(emd, sgd)
            inputs.append((plans[-1].render(emd, sgd, S), sgd))
        alone = []
        for p, (F, sig) in zip(plans, inputs):
            out = torch.zeros((3,) + p.vol_shape, device="cuda")
            p.reconstruct(F, sig, out, 4)
            alone.append(out)
        for p, (F, sig) in zip(plans, inputs):
            p.job_begin(F, sig, torch.zeros((3,) + p.vol_shape, device="cuda"))
        # four steps per plan; the first plan of a step (whose region stages the
        # in-scatter arguments) varies
        for group in ([0, 1], [2, 0, 3], [1, 2, 3, 0], [3, 1], [0, 2], [1, 3, 2]):
            rte().job_step([plans[i] for i in group])
        for i, (a, p) in enumerate(zip(alone, plans)):
            out = torch.empty((3,) + p.vol_shape, device="cuda")
            p.job_end(out)
            torch.cuda.synchronize()
            assert torch.equal(a, out), i
    finally:
        for p in plans:
            p.close()
