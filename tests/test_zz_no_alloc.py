"""The plan-free render (rte_render_static, for callers that cannot allocate
device memory) against the plan render it stands in for, through the C ABI:
bitwise the same images on consecutive calls that share the library's static
device array -- a large three-channel volume with in-scattering, then a
smaller ragged one-channel volume, a Henyey-Greenstein case with one
in-scatter grid per view, a rig whose rays all miss the box and cameras
inside the volume -- and no change of the device's free memory across
calls. The plan render itself is checked against the FP64 oracle elsewhere;
here the first case is also compared with the oracle directly."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import RENDER_REL, as64, dev, f32, host, render_rel, say

pytestmark = pytest.mark.gpu


def rte():
    from paper_1809_06417_amd import rte as _rte
    return _rte


def blobs(grid, C, seed, n_blobs=4):
    rng = np.random.default_rng(seed)
    lo, hi = np.array(grid.lo), np.array(grid.hi)
    ext = (hi - lo).min()
    centres = [lo + (hi - lo) * rng.uniform(0.25, 0.75, 3) for _ in range(n_blobs)]
    covs = [np.diag((ext * rng.uniform(0.08, 0.2, 3)) ** 2) for _ in range(n_blobs)]
    peaks = rng.uniform(0.4, 1.0, size=(n_blobs, C + 1))
    peaks[:, C] *= rng.uniform(1.0, 4.0) / ext
    f = synth.blob_fields(grid, centres, covs, peaks)
    return f32(f[:C]), f32(f[C])


CASES = {
    # 3 channels, isotropic in-scattering, 4 views 40x36 (ragged tiles)
    "colour": dict(grid=synth.Grid(40, 40, 40), views=4, W=40, H=36, C=3, albedo=0.3, M=8, dirs=16, g=0.0,
                   bg=0.05, seed=7),
    # smaller: non-cubic shifted box, 1 channel, 3 views 37x29
    "ragged": dict(grid=synth.Grid(13, 11, 9, lo=(-0.2, 0.1, 0.0), hi=(1.1, 0.9, 0.7)), views=3, W=37, H=29,
                   C=1, albedo=0.0, M=0, dirs=32, g=0.0, bg=0.0, seed=11),
    # Henyey-Greenstein in-scattering: one in-scatter grid per view
    "hg": dict(grid=synth.Grid(20, 18, 16), views=3, W=24, H=20, C=3, albedo=0.3, M=6, dirs=12, g=0.5,
               bg=0.0, seed=3),
    # every ray misses the box: the images are the background
    "miss": dict(grid=synth.Grid(12, 12, 12), views=2, W=16, H=12, C=3, albedo=0.0, M=0, dirs=32, g=0.0,
                 bg=0.25, seed=4, rig=dict(radius=1.0, centre=(6.0, 6.0, 6.0))),
    # cameras inside the volume
    "inside": dict(grid=synth.Grid(16, 16, 16), views=3, W=20, H=18, C=1, albedo=0.0, M=0, dirs=32, g=0.0,
                   bg=0.0, seed=5, rig=dict(radius=0.15, fov_y_deg=80.0)),
}


def inputs(name):
    c = CASES[name]
    g = c["grid"]
    rig = synth.ring_rig(c["views"], c["W"], c["H"], elevation_jitter_deg=12, seed=c["seed"], **c.get("rig", {}))
    em, sig = blobs(g, c["C"], c["seed"])
    return c, g, rig, em, sig


def plan_render(c, g, rig, em_d, sig_d):
    """The existing entry point: a plan, its in-scatter grid and its render."""
    with rte().Plan(g, rig, channels=c["C"], albedo=c["albedo"], background=c["bg"], scatter_res=c["M"],
                    scatter_dirs=c["dirs"], phase_g=c["g"]) as p:
        S = p.inscatter(em_d, sig_d) if c["albedo"] > 0 else None
        img = p.render(em_d, sig_d, S)
        return host(img), S


def static_render(c, g, rig, em_d, sig_d, S, out):
    return rte().render_static(g, rig, em_d, sig_d, S, channels=c["C"], albedo=c["albedo"], background=c["bg"],
                               scatter_res=c["M"], scatter_dirs=c["dirs"], phase_g=c["g"], out=out)


def test_static_render_equals_plan_render_on_consecutive_calls():
    import torch
    results = {}
    for name in ("colour", "ragged", "hg", "miss", "inside"):
        c, g, rig, em, sig = inputs(name)
        say("static render", name, g.nx, g.ny, g.nz, c["views"], c["W"], c["H"])
        em_d, sig_d = dev(em), dev(sig)
        ref, S = plan_render(c, g, rig, em_d, sig_d)
        out = torch.full((c["views"], c["C"], c["H"], c["W"]), float("nan"), device="cuda")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        static_render(c, g, rig, em_d, sig_d, S, out)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        got = host(out)
        assert np.isfinite(got).all(), name
        assert np.array_equal(got, ref), f"{name}: max |diff| {np.abs(got - ref).max():.3e}"
        results[name] = (free0, free1, got)
        if name == "colour":
            S64 = as64(host(S))
            F = oracle.render(g, rig, as64(em), as64(sig), step_vox=0.5, albedo=c["albedo"],
                              background=c["bg"], inscatter=S64)
            assert render_rel(got, F) <= RENDER_REL
        if name == "miss":
            assert np.all(got == np.float32(c["bg"]))
    # after the first call the array is resident: later calls change no free memory
    for name in ("ragged", "hg", "miss", "inside"):
        free0, free1, _ = results[name]
        assert free1 == free0, f"{name}: device free memory changed by {free0 - free1} bytes"


def test_static_render_repeats_after_a_larger_call():
    """The array keeps the last call's contents: a small render after a large
    one equals the small render done first."""
    import torch
    first = {}
    order = ("ragged", "colour", "ragged")
    for i, name in enumerate(order):
        c, g, rig, em, sig = inputs(name)
        say("static render sequence", i, name)
        em_d, sig_d = dev(em), dev(sig)
        S = None
        if c["albedo"] > 0:
            with rte().Plan(g, rig, channels=c["C"], albedo=c["albedo"], scatter_res=c["M"],
                            scatter_dirs=c["dirs"], phase_g=c["g"]) as p:
                S = p.inscatter(em_d, sig_d)
        out = torch.empty((c["views"], c["C"], c["H"], c["W"]), device="cuda")
        got = host(static_render(c, g, rig, em_d, sig_d, S, out))
        if name in first:
            assert np.array_equal(got, first[name])
        first[name] = got
