"""Throughput of the reconstruction hot path on one MI355X.

A step is one iteration of the reconstruction loop over the whole workload
(in-scatter grid, render of every view with the fused residual, voxel-owned
back-projection, update). Inputs are seeded synthetic volumes and camera
rings, resident in HBM before timing starts.

  python bench.py [--steps K] [--warmup W] [--workload colour|temperature|tiny|diff|serve]

Prints one JSON line. The metric is march samples per second (sum over all
pixel rays of their segment counts, times iterations, over wall time).

The serve workload is a stream of per-frame jobs (10 SART iterations each)
from six seeded flame videos arriving at Poisson times; there a step is one
job, --steps the number of jobs, and the line adds p50/p99 latency and
frames/s of the continuous-batching loop and of one job at a time.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per march sample (trilinear gathers of the render and the
# per-corner accumulation of the back-projection; no cache filtering).
#   render : 8 corners x (C emission + 1 extinction) x 4 B  [+ 8 x 12 B in-scatter grid]
#   gather : 8 corners x C accumulators x 4 B
def bytes_per_sample(C: int, scatter: bool):
    render = 8 * (C + 1) * 4 + (8 * 12 if scatter else 0)
    gather = 8 * C * 4
    return render, gather


WORKLOADS = {
    "colour": dict(n=128, views=8, W=512, H=512, C=3, albedo=0.3, M=32, dirs=32, iters=20),
    # the colour workload with Henyey-Greenstein in-scattering (g = 0.5, one
    # in-scatter grid per view)
    "colour_hg": dict(n=128, views=8, W=512, H=512, C=3, albedo=0.3, M=32, dirs=32, iters=20, phase_g=0.5),
    "temperature": dict(n=128, views=8, W=512, H=512, C=1, albedo=0.0, M=0, dirs=32, iters=30),
    "tiny": dict(n=32, views=4, W=64, H=64, C=1, albedo=0.0, M=0, dirs=32, iters=5),
    # gradient-based reconstruction: one step = forward march + adjoint march +
    # gradient gather + Adam update of (emission, extinction)
    "diff": dict(n=256, views=12, W=1024, H=768, C=3, albedo=0.3, M=32, dirs=32, iters=50),
    # grids, views and image sizes drawn per video (64-256^3, 4-12 views,
    # 256^2-1024x768), 3 channels, no scattering
    # the paper's extra evaluation (Sec. 5.1): 10 views 36 degrees apart at
    # 640x480, FOV 60, cameras 1.5 box lengths from the centre with +-10
    # degree elevations; grid from the volume-dimension rule (alpha = 1.5);
    # reconstruct from 9 views, measure the held-out one
    "lovo": dict(n=0, views=10, W=640, H=480, C=3, albedo=0.3, M=32, dirs=32, iters=20),
    # camera-count sweep of the temperature reconstruction (Sec. 5.2): rings of
    # 4, 16 and 28 cameras, 30 iterations each
    "sweep": dict(n=128, views=0, W=256, H=256, C=1, albedo=0.0, M=0, dirs=32, iters=30, counts=(4, 16, 28)),
    "serve": dict(n=0, views=0, W=0, H=0, C=3, albedo=0.0, M=0, dirs=32, iters=10,
                  videos=6, rate=40.0, sustainable_rate=12.0),
}


def inscatter_samples(n: int, M: int, ndirs: int, s_step: float = 0.5) -> int:
    """March samples of one in-scatter pass on an n^3 unit-cube grid: from each
    of the M^3 nodes along each spherical-Fibonacci direction to the box exit
    with steps of s_step coarse spacings (FP32, as the kernel counts them;
    a count may differ by one where a chord is a whole number of steps)."""
    import numpy as np
    k = np.arange(ndirs, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / ndirs
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    ph = k * np.pi * (3.0 - np.sqrt(5.0))
    h = 1.0 / (n - 1)
    u = np.stack([r * np.cos(ph), r * np.sin(ph), z], 1) / h          # voxel units per world unit
    u = u.astype(np.float32)
    scale = np.float32((n - 1) / (M - 1))
    p = (np.arange(M, dtype=np.float32) * scale).astype(np.float32)
    P = np.stack(np.meshgrid(p, p, p, indexing="ij"), -1).reshape(-1, 3)  # node coords (any axis order)
    top = np.float32(n - 1)
    ds = np.float32(s_step / (M - 1))
    total = 0
    for d in range(ndirs):
        ell = np.full(P.shape[0], np.inf, dtype=np.float32)
        for ax in range(3):
            ua = u[d, ax]
            if ua > 0:
                ell = np.minimum(ell, (top - P[:, ax]) / ua)
            elif ua < 0:
                ell = np.minimum(ell, -P[:, ax] / ua)
        ell = np.maximum(ell, np.float32(0.0))
        total += int(np.where(ell > 0, np.ceil(ell / ds), 0).sum())
    return total


def copy_bandwidth(gib: float = 2.0, reps: int = 5) -> float:
    """Achievable HBM bandwidth (GB/s, read + write) of a plain device copy of
    `gib` GiB, median of `reps` timed copies."""
    import torch
    n = int(gib * 2**30) // 4
    src = torch.empty(n, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    del src, dst
    torch.cuda.empty_cache()
    times.sort()
    return 2 * n * 4 / times[len(times) // 2] / 1e9


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("rte_kernels.hip",):
        h.update(open(os.path.join(ROOT, "paper_1809_06417_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def load_counters(kernel: str, workload: str):
    """Counter record of `kernel` on `workload` from the committed rocprofv3
    summary (profiles/<kernel>_<workload>_hbm_traffic.md): DRAM bytes per
    launch (calibrated FETCH_SIZE + WRITE_SIZE) and, where measured, the
    texture data path busy fraction. None when absent or measured on a
    different kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\s*(\{.*?\})\s*```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("kernel_source_sha") != kernel_source_sha():
        return None
    return rec


def compulsory_floor(n_nodes: int, C: int, views: int, W: int, H: int) -> int:
    """Bytes an iteration must move at least: the packed volume (emission +
    extinction) read once per view, the frames read once and the volume update
    written once."""
    elem = 16 if C == 3 else 8
    return views * n_nodes * elem + views * C * H * W * 4 + C * n_nodes * 4


def roofline_record(dom: str, avg_s: float, alg_bytes: int, n_units: int, workload: str, launches: int,
                    all_kernels: dict, achievable=None, floor=None):
    """Roofline of the dominant kernel: DRAM bytes per launch (from the
    committed counter summary) over its live average launch duration, against
    the HBM peak. The method's logical bytes per launch (trilinear gathers and
    per-corner accumulations, served mostly from registers, LDS and caches)
    are reported beside it under `algorithmic`, never as `frac`."""
    rec = load_counters(dom, workload)
    traffic = float(rec["hbm_bytes_per_launch"]) if rec else None
    dram = traffic / avg_s / 1e9 if traffic else None
    out = {"bound": "hbm", "achieved": round(dram, 1) if dram else None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(dram / HBM_PEAK_GBS, 4) if dram else None, "traffic": traffic, "kernel": dom,
           "avg_ms": round(avg_s * 1e3, 4), "launches": launches,
           "algorithmic": {"bytes_per_sample": alg_bytes // max(n_units, 1), "samples_per_launch": n_units,
                           "GBs": round(alg_bytes / avg_s / 1e9, 1)}}
    if rec and rec.get("td_busy") is not None:
        out["onchip"] = {"bound": "texture data path", "busy": rec["td_busy"], "peak": 1.0,
                         "unit": "busy cycles per cycle (rocprofv3 TD_TD_BUSY)"}
    if floor:
        out["floor_bytes_per_iteration"] = floor
        if traffic:
            out["traffic_over_floor"] = round(traffic / floor, 3)
    if achievable:
        out["achievable_copy_GBs"] = round(achievable, 1)
    out["all"] = all_kernels
    return out


def step_spread(step_fn, fresh, steps, repeats):
    """The timed steps run again `repeats` times (each from the same start,
    after the main measurement): median and 5th/95th percentiles of the time
    per step over the repeats. Reported beside `ms_per_step`, never in place
    of it."""
    import numpy as np
    import torch
    if repeats <= 0:
        return None
    per_step = []
    for _ in range(repeats):
        x = fresh()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step_fn(x, steps)
        torch.cuda.synchronize()
        per_step.append((time.perf_counter() - t0) / steps * 1e3)
    q = np.percentile(per_step, [5, 50, 95])
    return {"repeats": repeats, "steps_each": steps, "p5": round(float(q[0]), 4), "p50": round(float(q[1]), 4),
            "p95": round(float(q[2]), 4)}


def max_rel(a, b):
    """max |a - b| / max |b| (0 when b is all zero)."""
    import numpy as np
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    scale = float(np.abs(b).max()) if b.size else 0.0
    return float(np.abs(a - b).max() / scale) if scale > 0 else 0.0


def cpu_baseline(g, rig, em, sig, frames, wl, views, gpu=None):
    """The FP64 oracle (as it stands) on a bounded sample: one iteration of the
    same loop (in-scatter grid, render, back-projection) restricted to the
    first `views` views. `gpu` (optional) holds the GPU's in-scatter grid and a
    back-projection callable; after the timing, the GPU results on the same
    inputs are compared with the oracle's (`accuracy`)."""
    import numpy as np

    import oracle
    sub = rig.subset(range(views))
    em64, sig64 = np.asarray(em, np.float64), np.asarray(sig, np.float64)
    F = np.asarray(frames[:views], np.float64)
    _, _, K = oracle.ray_table(g, sub, 0.5)
    samples = int(K.sum())
    t0 = time.perf_counter()
    S = None
    if wl["albedo"] > 0:
        S = oracle.inscatter(g, em64, sig64, s_res=wl["M"], n_dirs=wl["dirs"], phase_g=wl.get("phase_g", 0.0),
                             rig=sub)
    I, R = oracle.render(g, sub, em64, sig64, albedo=wl["albedo"], inscatter=S, rowsum=True)
    y = np.where(R[:, None] > 0, (F - I) / np.where(R[:, None] > 0, R[:, None], 1.0), 0.0)
    oracle.backproject_adjoint(g, sub, sig64, y)
    dt = time.perf_counter() - t0
    out = dict(value=samples / dt, unit="samples/s", cores=oracle.num_threads(), kind="oracle",
               sample=f"one FP64 iteration (in-scatter grid, render, back-projection) on "
                      f"{views} of {rig.n_views} views: {samples} samples in {dt:.1f} s",
               cpu=cpu_model())
    # the same on one thread, over one view (the in-scatter grid is computed in full)
    threads = oracle.num_threads()
    one = rig.subset([0])
    _, _, K1 = oracle.ray_table(g, one, 0.5)
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        S1 = None
        if wl["albedo"] > 0:
            S1 = oracle.inscatter(g, em64, sig64, s_res=wl["M"], n_dirs=wl["dirs"], phase_g=wl.get("phase_g", 0.0),
                                  rig=one)
        I1, R1 = oracle.render(g, one, em64, sig64, albedo=wl["albedo"], inscatter=S1, rowsum=True)
        y1 = np.where(R1[:, None] > 0, (F[:1] - I1) / np.where(R1[:, None] > 0, R1[:, None], 1.0), 0.0)
        oracle.backproject_adjoint(g, one, sig64, y1)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(threads)
    out["single_thread"] = dict(value=int(K1.sum()) / dt1, unit="samples/s",
                                sample=f"one view: {int(K1.sum())} samples in {dt1:.1f} s (in-scatter grid included)")
    if gpu is not None:
        # accuracy beside speed: the GPU's frames (its render of the benchmark's
        # inputs) against the oracle's render, per view and channel; its
        # in-scatter grid; and both back-projections of one FP32 residual
        acc = {"render_max_rel_err": max(max_rel(frames[v, c], I[v, c]) for v in range(views)
                                         for c in range(I.shape[1]))}
        if S is not None and gpu.get("S") is not None and np.shape(gpu["S"]) == np.shape(S):
            acc["inscatter_max_rel_err"] = max_rel(gpu["S"], S)
        y32 = y.astype(np.float32)
        d_orc = oracle.backproject_adjoint(g, sub, sig64, y32.astype(np.float64))
        acc["backproject_max_rel_err"] = max_rel(gpu["backproject"](y32), d_orc)
        acc["note"] = (f"GPU against the FP64 oracle on the benchmark's inputs, {views} of {rig.n_views} views; "
                       f"relative to the oracle's largest value")
        out["accuracy"] = acc
    return out


def cpu_baseline_temperature(g, rig, frames, gpu_T1=None):
    """The FP64 oracle's temperature fit (as it stands), one iteration from
    800 K on all views of the temperature workload (colour-temperature map,
    render of the fitted channel with row sums, back-projection with column
    sums, EM update, LUT inverse); `gpu_T1` (optional), the GPU's result of the
    same iteration, is compared with it."""
    import numpy as np

    import oracle
    tp = oracle.TempParams()
    lut = oracle.temp_lut(tp)
    F = np.asarray(frames, np.float64)
    _, _, K = oracle.ray_table(g, rig, 0.5)
    samples = int(K.sum())
    T0 = np.full(g.shape_zyx, 800.0)
    t0 = time.perf_counter()
    T1 = oracle.temperature_fit(g, rig, tp, lut, F, T0, 1)
    dt = time.perf_counter() - t0
    out = dict(value=samples / dt, unit="samples/s", cores=oracle.num_threads(), kind="oracle",
               sample=f"one FP64 iteration of the temperature fit on {rig.n_views} of {rig.n_views} views: "
                      f"{samples} samples in {dt:.1f} s", cpu=cpu_model())
    if gpu_T1 is not None:
        d = np.abs(np.asarray(gpu_T1, np.float64) - T1)
        out["accuracy"] = {"temperature_max_abs_err_K": float(d.max()),
                           "temperature_rms_err_K": float(np.sqrt((d ** 2).mean())),
                           "note": "GPU against the FP64 oracle after one iteration from 800 K on the "
                                   "benchmark's frames"}
    return out


def cpu_baseline_diff(g, rig, em0, sig0, S, frames, gpu_grad=None):
    """The FP64 oracle's gradient (as it stands) on a bounded sample of the
    differentiable workload: the loss 1/2 |I - F|^2 over view 0 only, at the
    timed steps' starting point, forward render plus gradient with respect to
    emission and extinction (the in-scatter grid held fixed, the GPU's, as in
    the timed steps). `gpu_grad(dLdI)` (optional) gives the GPU's gradients of
    the same loss for comparison."""
    import numpy as np

    import oracle
    one = rig.subset([0])
    em64, sig64 = np.asarray(em0, np.float64), np.asarray(sig0, np.float64)
    S64 = np.asarray(S, np.float64)
    F = np.asarray(frames[:1], np.float64)
    _, _, K = oracle.ray_table(g, one, 0.5)
    samples = int(K.sum())
    kw = dict(step_vox=0.5, albedo=0.3, inscatter=S64)
    t0 = time.perf_counter()
    I = oracle.render(g, one, em64, sig64, **kw)
    dLdI = I - F
    d_em, d_sig = oracle.render_grad(g, one, em64, sig64, dLdI, **kw)
    dt = time.perf_counter() - t0
    out = dict(value=samples / dt, unit="samples/s", cores=oracle.num_threads(), kind="oracle",
               sample=f"one FP64 forward render and gradient on 1 of {rig.n_views} views: "
                      f"{samples} samples in {dt:.1f} s", cpu=cpu_model())
    if gpu_grad is not None:
        ge, gs = gpu_grad(dLdI.astype(np.float32))
        out["accuracy"] = {"grad_emission_max_rel_err": max_rel(ge, d_em),
                           "grad_extinction_max_rel_err": max_rel(gs, d_sig),
                           "note": "GPU against the FP64 oracle, same loss, view 0, relative to the oracle's "
                                   "largest gradient"}
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip() + f" ({os.cpu_count()} logical CPUs visible)"
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="iterations (jobs for serve); default 20 (300)")
    ap.add_argument("--warmup", type=int, default=20,
                    help="untimed steps first; fewer than about 20 leave the GPU short of its steady clocks")
    ap.add_argument("--workload", default="colour", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-views", type=int, default=8, help="views in the CPU baseline sample (one FP64 iteration)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--repeats", type=int, default=5,
                    help="after the timed steps: time the same steps again this many times for the spread")
    ap.add_argument("--hbm-budget-gib", type=int, default=64, help="serve: workspace budget for resident plans")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (HBM counter scale)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 300 if args.workload == "serve" else 20
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * 2**20 // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design "
              f"(view sharding + one all-reduce per iteration) is not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1809_06417_amd import rte

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    wl = WORKLOADS[args.workload]
    if args.workload == "serve":
        return run_serve(args, wl)
    if args.workload == "lovo":
        return run_lovo(args, wl)
    if args.workload == "sweep":
        return run_sweep(args, wl)
    print(f"[bench] workload {args.workload}: building inputs", file=sys.stderr, flush=True)
    if args.workload in ("colour", "colour_hg", "diff"):
        g, em, sig = synth.colour_volume(args.seed, n=wl["n"])
    elif args.workload == "tiny":
        g, em, sig = synth.tiny_volume(args.seed, n=wl["n"])
    else:
        g, T = synth.temperature_volume(args.seed, n=wl["n"])
    rig = synth.ring_rig(wl["views"], wl["W"], wl["H"])
    C = wl["C"]
    plan = rte.Plan(g, rig, channels=C, step_vox=0.5, albedo=wl["albedo"],
                    scatter_res=wl["M"], scatter_dirs=wl["dirs"], gradients=args.workload == "diff",
                    phase_g=wl.get("phase_g", 0.0))
    dev = lambda a: torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")
    if args.workload == "temperature":
        tp = rte.TempParams()
        Td = dev(T)
        em3, sg = plan.temperature_map(Td, tp)
        frames = torch.zeros((wl["views"], 3, wl["H"], wl["W"]), device="cuda")
        frames[:, 1] = plan.render(em3[1:2].contiguous(), sg)[:, 0]
        x0 = torch.full_like(Td, 800.0)
        step_fn = lambda x, k: plan.reconstruct_temperature(frames, x, k, tp)
    elif args.workload == "diff":
        from paper_1809_06417_amd import autograd
        emd, sigd = dev(em), dev(sig)
        S = plan.inscatter(emd, sigd)
        frames = plan.render(emd, sigd, S)
        x0 = (torch.full_like(emd, 0.1), torch.full_like(sigd, 0.5))

        def step_fn(x, k):
            em_p, sg_p = x[0].requires_grad_(True), x[1].requires_grad_(True)
            # the fused form runs the whole update in one kernel per step
            opt = torch.optim.Adam([em_p, sg_p], lr=0.02, fused=True)
            for _ in range(k):
                opt.zero_grad(set_to_none=False)
                loss = 0.5 * ((autograd.render(plan, em_p, sg_p, S) - frames) ** 2).sum()
                loss.backward()
                opt.step()
                with torch.no_grad():
                    em_p.clamp_(min=0.0)
                    sg_p.clamp_(min=0.0)
            return em_p
    else:
        emd, sigd = dev(em), dev(sig)
        S = plan.inscatter(emd, sigd) if wl["albedo"] > 0 else None
        frames = plan.render(emd, sigd, S)
        x0 = torch.zeros_like(emd)
        step_fn = lambda x, k: plan.reconstruct(frames, sigd, x, k)
    torch.cuda.synchronize()
    print(f"[bench] plan: {plan.samples} samples/iteration, {plan.hit_rays} hit rays, "
          f"{plan.device_bytes / 2**20:.0f} MiB workspace", file=sys.stderr, flush=True)

    fresh = (lambda: tuple(t.clone() for t in x0)) if isinstance(x0, tuple) else (lambda: x0.clone())
    samples = plan.samples
    b_render, b_gather = bytes_per_sample(C, wl["albedo"] > 0)
    # algorithmic bytes per launch of each candidate kernel
    cands = {"render": b_render * samples, "gather": b_gather * samples}
    if args.workload == "diff":
        # the adjoint march re-reads what the render reads; the gradient gather
        # accumulates C emission + 1 extinction values per corner
        cands = {"render": b_render * samples, "adjoint": b_render * samples,
                 "gather": 8 * (C + 1) * 4 * samples}
    scat_samples = None
    if wl["albedo"] > 0 and wl["M"] >= 2:
        # in-scatter march: 8 corners x 16 B (packed RGB + extinction) per sample
        scat_samples = inscatter_samples(wl["n"], wl["M"], wl["dirs"])
        cands["inscatter"] = 8 * 16 * scat_samples

    # warmup with every kernel timed, which names the dominant kernel
    x = fresh()
    dom = None
    if args.warmup > 0:
        plan.set_timing(True)
        step_fn(x, args.warmup)
        torch.cuda.synchronize()
        wt = {k: plan.kernel_time(k) for k in cands}
        plan.set_timing(False)
        dom = max(cands, key=lambda k: wt[k][0])
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    # the timed region: only the dominant kernel's launches carry events (each
    # event adds a marker of a few microseconds to the stream); with no warmup
    # every kernel is timed
    x = fresh()
    plan.set_timing(True, kernels=[dom] if dom else None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_fn(x, args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ktimes = {k: plan.kernel_time(k) for k in rte.KERNELS}
    plan.set_timing(False)
    print(f"[bench] timed {args.steps} steps in {elapsed * 1e3:.1f} ms", file=sys.stderr, flush=True)
    if dom is None:
        dom = max(cands, key=lambda k: ktimes[k][0])
    # per-kernel table: the same steps once more, every kernel timed
    table = ktimes
    if args.warmup > 0:
        x = fresh()
        plan.set_timing(True)
        step_fn(x, args.steps)
        torch.cuda.synchronize()
        table = {k: plan.kernel_time(k) for k in rte.KERNELS}
        plan.set_timing(False)
    spread = step_spread(step_fn, fresh, args.steps, args.repeats)

    value = samples * args.steps / elapsed
    per_kernel = {}
    for k, (ms, n) in table.items():
        if n:
            per_kernel[k] = {"avg_ms": ms / n, "launches": n, "total_ms": ms}
    dom_avg_s = ktimes[dom][0] / max(ktimes[dom][1], 1) / 1e3
    n_units = scat_samples if dom == "inscatter" else samples
    achievable = copy_bandwidth()
    all_k = {}
    for k, v in cands.items():
        if not table[k][1]:
            continue
        avg = table[k][0] / table[k][1] / 1e3
        rec = load_counters(k, args.workload)
        all_k[k] = {"avg_ms": round(avg * 1e3, 4), "algorithmic_GBs": round(v / avg / 1e9, 1),
                    "dram_GBs": round(float(rec["hbm_bytes_per_launch"]) / avg / 1e9, 1) if rec else None}
    floor = compulsory_floor(g.nx * g.ny * g.nz, C, wl["views"], wl["W"], wl["H"])
    roofline = roofline_record(dom, dom_avg_s, cands[dom], n_units, args.workload, ktimes[dom][1], all_k,
                               achievable, floor)

    base = None
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a bounded sample", file=sys.stderr, flush=True)
        if args.workload == "diff":
            from paper_1809_06417_amd import autograd
            em0, sg0 = (t.detach().cpu().numpy() for t in x0)

            def gpu_grad(dldi0):
                e = x0[0].clone().requires_grad_(True)
                sg = x0[1].clone().requires_grad_(True)
                img = autograd.render(plan, e, sg, S)
                (img[0] * torch.from_numpy(dldi0[0]).cuda()).sum().backward()
                torch.cuda.synchronize()
                return e.grad.cpu().numpy(), sg.grad.cpu().numpy()

            base = cpu_baseline_diff(g, rig, em0, sg0, S.cpu().numpy(), frames.cpu().numpy(), gpu_grad)
        elif args.workload == "temperature":
            x1 = x0.clone()
            plan.reconstruct_temperature(frames, x1, 1, tp)
            torch.cuda.synchronize()
            base = cpu_baseline_temperature(g, rig, frames.cpu().numpy(), x1.cpu().numpy())
        else:
            nv = min(args.cpu_views, wl["views"])

            def gpu_backproject(y32):
                # the plan back-projects every view: the views outside the sample get 0
                full = np.zeros((wl["views"],) + y32.shape[1:], np.float32)
                full[:nv] = y32
                d = plan.backproject(sigd, torch.from_numpy(full).cuda())
                torch.cuda.synchronize()
                return d.cpu().numpy()

            gpu = {"S": S.cpu().numpy() if S is not None else None, "backproject": gpu_backproject}
            base = cpu_baseline(g, rig, em, sig, frames.cpu().numpy(), wl, nv, gpu)

    out = {
        "metric": "ray samples/s per render+backproject iteration",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl['n']}^3 grid, {C} channel(s), "
                               f"{wl['views']} views of {wl['W']}x{wl['H']}, step 0.5 voxel, "
                               f"albedo {wl['albedo']}" + (f", in-scatter {wl['M']}^3 x {wl['dirs']} dirs"
                                                           if wl["M"] else "")
                               + (f", Henyey-Greenstein g = {wl['phase_g']} (one in-scatter grid per view)"
                                  if wl.get("phase_g") else ""),
                   "samples_per_step": samples, "hit_rays": plan.hit_rays,
                   "frames_per_s": args.steps / elapsed / wl["iters"]},
        "roofline": roofline,
        "cpu_baseline": base,
        "step_ms_spread": spread,
        "kernels": per_kernel,
    }
    print(json.dumps(out))
    plan.close()


def run_lovo(args, wl):
    """Leave-one-view-out evaluation; a step is one reconstruction iteration
    over the nine input views."""
    import torch

    import synth
    from paper_1809_06417_amd import evaluate, rte

    rig = synth.ring_rig(wl["views"], wl["W"], wl["H"], radius=1.5, fov_y_deg=60.0, elevation_jitter_deg=10.0,
                         seed=args.seed)
    (nx, ny, nz), nmax = rte.suggest_grid(rig, alpha=1.5)
    g = synth.Grid(nx, ny, nz)
    print(f"[bench] lovo: grid {nx}x{ny}x{nz} from projected edges {nmax}", file=sys.stderr, flush=True)
    fields = synth.blob_fields_torch(g, *synth.colour_blobs(args.seed), device="cuda")
    em, sig = fields[:3].contiguous(), fields[3].contiguous()
    kw = dict(step_vox=1.0, albedo=wl["albedo"], scatter_res=wl["M"], scatter_dirs=wl["dirs"])
    evaluate.leave_one_view_out(g, rig, em, sig, wl["views"] - 1, max(args.warmup, 1), **kw)  # warm-up
    r = evaluate.leave_one_view_out(g, rig, em, sig, wl["views"] - 1, args.steps, timing=True, **kw)
    samples = r["samples_per_iter"]
    value = samples * args.steps / r["reconstruct_s"]
    b_render, b_gather = bytes_per_sample(wl["C"], True)
    ms, n = r["kernels"]["render"]
    achieved = b_render * samples / (ms / n / 1e3) / 1e9
    out = {
        "metric": "ray samples/s per render+backproject iteration", "value": value, "unit": "samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["reconstruct_s"] / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"lovo: colour plume volume on the {nx}x{ny}x{nz} grid the volume-dimension "
                               f"rule gives (alpha 1.5), 10 views 640x480 FOV 60 at 1.5 box lengths, step "
                               f"1 voxel, albedo 0.3, in-scatter 32^3; {args.steps} SART iterations from "
                               f"zero on 9 views, view 9 held out", "samples_per_step": samples},
        "evaluation": {"pixel_rmse_input_rgb": [round(float(v), 3) for v in r["input"]],
                       "pixel_rmse_test_rgb": [round(float(v), 3) for v in r["test"]],
                       "volume_rmse_rgb": [round(float(v), 3) for v in r["volume"]],
                       "scale": "0-255 (frames' maximum = 255)"},
        "roofline": roofline_record("render", ms / n / 1e3, b_render * samples, samples, "lovo", n,
                                    {"render": {"avg_ms": round(ms / n, 4),
                                                "algorithmic_GBs": round(achieved, 1)}}),
        "cpu_baseline": None,
        "kernels": {k: {"avg_ms": ms_ / n_, "launches": n_} for k, (ms_, n_) in r["kernels"].items() if n_},
    }
    print(json.dumps(out))


def run_sweep(args, wl):
    """Camera-count sweep of the temperature fit; a step is one fit iteration,
    summed over the rigs."""
    import torch

    import synth
    from paper_1809_06417_amd import evaluate

    g, T = synth.temperature_volume(args.seed, n=wl["n"])
    Td = torch.tensor(T.astype("float32"), device="cuda")
    rigs = [synth.ring_rig(n, wl["W"], wl["H"], elevation_jitter_deg=10.0, seed=args.seed) for n in wl["counts"]]
    evaluate.camera_sweep(g, Td, rigs[:1], 2)  # warm-up
    res = evaluate.camera_sweep(g, Td, rigs, wl["iters"])
    samples = sum(r["samples_per_iter"] for r in res)
    secs = sum(r["reconstruct_s"] for r in res)
    value = samples * wl["iters"] / secs
    out = {
        "metric": "ray samples/s per render+backproject iteration", "value": value, "unit": "samples/s",
        "n_gpus": 1, "steps": wl["iters"] * len(rigs), "warmup": 2,
        "ms_per_step": secs / (wl["iters"] * len(rigs)) * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"sweep: temperature fit on the {wl['n']}^3 plume field with rings of "
                               f"{', '.join(str(n) for n in wl['counts'])} cameras at {wl['W']}x{wl['H']}, "
                               f"{wl['iters']} iterations from 800 K each"},
        "evaluation": [{"cameras": r["cameras"], "pixel_rmse_rgb": [round(float(v), 3) for v in r["image"]],
                        "temperature_rmse_K": round(r["temperature_K"], 2), "hull_voxels": r["voxels"],
                        "seconds": round(r["reconstruct_s"], 4)} for r in res],
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out))


def run_serve(args, wl):
    """Serving: jobs arrive at Poisson times; the continuous-batching loop runs
    them, then the same jobs run one at a time for comparison. Both are run at
    the offered rate and at a sustainable rate below either path's capacity."""
    import numpy as np
    import torch

    import synth
    from paper_1809_06417_amd import rte, serve

    n_jobs = args.steps
    vids = np.random.default_rng([args.seed, 1]).integers(0, wl["videos"], size=n_jobs)
    specs = {v: synth.video_spec(v, seed=args.seed) for v in range(wl["videos"])}
    print(f"[bench] serve: {n_jobs} jobs, {wl['videos']} videos, generating frames", file=sys.stderr, flush=True)
    inputs, frame_of = {}, []
    count = {}
    samples_of = {}
    for v, spec in specs.items():
        with rte.Plan(spec.grid, spec.rig, channels=wl["C"]) as p:
            samples_of[v] = p.samples
            nf = int((vids == v).sum())
            for fr in range(nf):
                em, sig = synth.video_frame(spec, fr, device="cuda")
                inputs[(v, fr)] = (p.render(em, sig), sig)
            torch.cuda.synchronize()
    for v in vids:
        fr = count.get(int(v), 0)
        count[int(v)] = fr + 1
        frame_of.append(fr)
    input_bytes = sum(F.numel() * 4 + s_.numel() * 4 for F, s_ in inputs.values())
    print(f"[bench] inputs: {input_bytes / 2**30:.1f} GiB resident", file=sys.stderr, flush=True)

    def make_jobs(arrivals):
        return [serve.Job(i, int(v), frame_of[i], float(t), *inputs[(int(v), frame_of[i])])
                for i, (t, v) in enumerate(zip(arrivals, vids))]

    budget = args.hbm_budget_gib << 30
    videos = {v: serve.VideoState(s, channels=wl["C"]) for v, s in specs.items()}
    # warmup: one job per video through the batched path (loads the kernels)
    warm = [serve.Job(i, v, 0, 0.0, *inputs[(v, 0)]) for i, v in enumerate(sorted(set(int(x) for x in vids)))]
    serve.serve(videos, warm, iters=min(args.warmup, wl["iters"]) or 1, hbm_budget_bytes=budget)

    def reset(vs_map):
        for vs in vs_map.values():
            vs.volume = None
            vs.resident = False
            vs.busy = False
        torch.cuda.synchronize()

    total_samples = sum(samples_of[int(v)] for v in vids) * wl["iters"]
    mean_job = float(np.mean([samples_of[int(v)] for v in vids])) * wl["iters"]
    runs = {}
    ktimes = {k: [0.0, 0] for k in rte.KERNELS}
    seq_videos = {v: serve.VideoState(s, channels=wl["C"]) for v, s in specs.items()}
    for label, rate in (("offered", wl["rate"]), ("sustainable", wl["sustainable_rate"])):
        arrivals = synth.poisson_arrivals(n_jobs, rate, seed=args.seed)
        reset(videos)
        timed = label == "offered"
        if timed:
            for vs in videos.values():
                if vs.plan is not None:
                    vs.plan.set_timing(True)
        print(f"[bench] serving at {rate:g} jobs/s", file=sys.stderr, flush=True)
        st = {}
        jobs = serve.serve(videos, make_jobs(arrivals), iters=wl["iters"], hbm_budget_bytes=budget,
                           log=lambda m: None, stats=st)
        torch.cuda.synchronize()
        summ = serve.latency_summary(jobs)
        summ["gpu_busy"] = round(st["gpu_busy"], 4)
        summ["samples_per_s"] = total_samples / summ["span_s"]
        summ["served_over_offered"] = round(summ["samples_per_s"] / (mean_job * rate), 4)
        if timed:
            for vs in videos.values():
                if vs.plan is not None:
                    for k in rte.KERNELS:
                        ms, n = vs.plan.kernel_time(k)
                        ktimes[k][0] += ms
                        ktimes[k][1] += n
                    vs.plan.set_timing(False)
        print(f"[bench] batched at {rate:g}/s: {summ}", file=sys.stderr, flush=True)
        reset(seq_videos)
        print(f"[bench] one job at a time at {rate:g} jobs/s", file=sys.stderr, flush=True)
        seq = serve.serve_sequential(seq_videos, make_jobs(arrivals), iters=wl["iters"])
        seq_summ = serve.latency_summary(seq)
        seq_summ["samples_per_s"] = total_samples / seq_summ["span_s"]
        seq_summ["served_over_offered"] = round(seq_summ["samples_per_s"] / (mean_job * rate), 4)
        print(f"[bench] sequential at {rate:g}/s: {seq_summ}", file=sys.stderr, flush=True)
        runs[label] = {"rate_jobs_per_s": rate, "offered_samples_per_s": mean_job * rate,
                       "batched": summ, "one_at_a_time": seq_summ}
    plans_resident = sum(vs.plan is not None for vs in videos.values())
    for vs in list(videos.values()) + list(seq_videos.values()):
        vs.evict()

    summ = runs["offered"]["batched"]
    value = summ["samples_per_s"]
    b_render, b_gather = bytes_per_sample(wl["C"], False)
    cands = {"render": b_render, "gather": b_gather}
    dom = max(cands, key=lambda k: ktimes[k][0])
    # aggregated over every batched launch: algorithmic bytes / kernel time
    avg_s = ktimes[dom][0] / max(ktimes[dom][1], 1) / 1e3
    roofline = roofline_record(dom, avg_s, cands[dom] * total_samples // max(ktimes[dom][1], 1),
                               total_samples // max(ktimes[dom][1], 1), "serve", ktimes[dom][1], {})
    roofline["kernel"] = dom + " (batched)"
    per_kernel = {k: {"avg_ms": ms / n, "launches": n, "total_ms": ms} for k, (ms, n) in ktimes.items() if n}
    out = {
        "metric": "ray samples/s per render+backproject iteration",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": n_jobs,
        "warmup": len(warm),
        "ms_per_step": summ["span_s"] / n_jobs * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"serve: {n_jobs} frame jobs from {wl['videos']} seeded videos "
                               f"(grids 64-256^3, 4-12 views, 256^2-1024x768, RGB, no scattering), "
                               f"Poisson arrivals at {wl['rate']:g} jobs/s (and at {wl['sustainable_rate']:g} "
                               f"jobs/s), {wl['iters']} SART iterations per job warm-started from the "
                               f"resident previous volume; batched loop on 2 stream lanes, 2 steps queued each, "
                               f"a waiting job sharing the GPU with running ones once 3 wait",
                   "videos": {v: f"{s.grid.nx}^3, {s.rig.n_views} views of {s.rig.width}x{s.rig.height}, "
                                 f"{samples_of[v]} samples/iteration" for v, s in specs.items()},
                   "hbm_budget_gib": args.hbm_budget_gib, "plans_resident": plans_resident,
                   "offered_samples_per_s": mean_job * wl["rate"],
                   "utilisation": summ["served_over_offered"]},
        "serving": runs,
        "roofline": roofline,
        "cpu_baseline": None,
        "kernels": per_kernel,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
