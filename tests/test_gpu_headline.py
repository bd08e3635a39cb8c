"""GPU parity at the full-size workloads the benchmark times, on the same
seeded inputs, against the FP64 oracle (Sec. 3.3; render tolerance per view
and channel, reconstruction tolerance after the fixed iteration counts).

* colour: 128^3 RGB emission + extinction from 20 plume blobs, 8 ring views
  of 512x512, albedo 0.3, isotropic in-scattering on a 32^3 grid with 32
  directions; the render of the true volume, then 20 SART iterations from
  zero against the oracle's frames.
* temperature: 128^3 temperature field, 8 views of 512x512, 30 iterations of
  the temperature fit from 800 K against the oracle's frames.
* the colour workload with Henyey-Greenstein in-scattering (g = 0.5): every
  view's in-scatter grid and render.
* the differentiable workload's forward model: 256^3 RGB + extinction with
  single scattering, 12 views of 1024x768: in-scatter grid and render.

The oracle needs a few seconds per iteration on the host's cores, so each
long run is cut into chunks of iterations (one test each, sharing the state
of the chunks before it; a chunk run on its own first runs the earlier
ones). Both loops carry no state between iterations other than the volume
(the SART sums and the in-scatter grid are recomputed from it, the
temperature fit re-derives everything from T), so ten iterations twice equal
twenty on either side."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import RENDER_REL, VOLUME_RMS, as64, dev, f32, host, rel_rms, render_rel, say

pytestmark = pytest.mark.gpu

STEP = 0.5
N, VIEWS, W, H = 128, 8, 512, 512
ALBEDO, M, DIRS = 0.3, 32, 32


def rte():
    from paper_1809_06417_amd import rte as _rte
    return _rte


_ST = {}


def colour():
    if "colour" not in _ST:
        g, em, sig = synth.colour_volume(0, n=N)
        rig = synth.ring_rig(VIEWS, W, H)
        em, sig = f32(em), f32(sig)
        S = oracle.inscatter(g, as64(em), as64(sig), s_res=M, n_dirs=DIRS)
        F = f32(oracle.render(g, rig, as64(em), as64(sig), step_vox=STEP, albedo=ALBEDO, inscatter=S))
        _ST["colour"] = dict(g=g, rig=rig, em=em, sig=sig, S=f32(S), F=F)
    return _ST["colour"]


def colour_plan(c):
    return rte().Plan(c["g"], c["rig"], channels=3, step_vox=STEP, albedo=ALBEDO, scatter_res=M,
                      scatter_dirs=DIRS)


def test_colour_workload_render_and_inscatter_match_oracle():
    c = colour()
    say("headline colour render")
    with colour_plan(c) as p:
        S = host(p.inscatter(dev(c["em"]), dev(c["sig"])))
        img = host(p.render(dev(c["em"]), dev(c["sig"]), dev(c["S"])))
    # in-scatter grid of the true volume, then the render with the oracle's
    # grid: every view and channel
    assert np.abs(S - c["S"]).max() / np.abs(c["S"]).max() <= RENDER_REL
    assert render_rel(img, c["F"]) <= RENDER_REL


def advance_colour(upto):
    """Run both sides on to `upto` SART iterations, 10 at a time, and check
    parity per channel at each chunk's end."""
    c = colour()
    while c.get("iters", 0) < upto:
        x_o = c.get("x_o", np.zeros((3, N, N, N)))
        x_g = c.get("x_g", np.zeros((3, N, N, N), dtype=np.float32))
        x_o = oracle.reconstruct(c["g"], c["rig"], as64(c["F"]), as64(c["sig"]), x_o, 10, step_vox=STEP,
                                 albedo=ALBEDO, s_res=M, n_dirs=DIRS)
        say("headline colour SART", c.get("iters", 0) + 10)
        with colour_plan(c) as p:
            xg = dev(x_g)
            p.reconstruct(dev(c["F"]), dev(c["sig"]), xg, 10)
            x_g = xg.cpu().numpy()
        c.update(x_o=x_o, x_g=x_g, iters=c.get("iters", 0) + 10)
        for ch in range(3):
            assert rel_rms(as64(x_g[ch]), x_o[ch]) <= VOLUME_RMS, (c["iters"], ch)


@pytest.mark.parametrize("upto", [10, 20])
def test_colour_workload_sart_matches_oracle(upto):
    advance_colour(upto)


def temperature():
    if "temp" not in _ST:
        g, T = synth.temperature_volume(0, n=N)
        rig = synth.ring_rig(VIEWS, W, H)
        T = f32(T)
        tp = oracle.TempParams()
        lut = oracle.temp_lut(tp)
        em, sig = oracle.temp_map(tp, lut, as64(T))
        F = np.zeros((VIEWS, 3, H, W), dtype=np.float32)
        F[:] = f32(oracle.render(g, rig, em, sig, step_vox=STEP))
        _ST["temp"] = dict(g=g, rig=rig, T=T, tp=tp, lut=lut, F=F)
    return _ST["temp"]


def advance_temperature(upto):
    """Run both fits on to `upto` iterations, 15 at a time; at each chunk's
    end compare the green emission of both fits (the observable) and the
    normalised temperature where the green emission is above 1e-3 of its
    maximum."""
    t = temperature()
    while t.get("iters", 0) < upto:
        T_o = t.get("T_o", np.full((N, N, N), 800.0))
        T_g = t.get("T_g", np.full((N, N, N), 800.0, dtype=np.float32))
        T_o = oracle.temperature_fit(t["g"], t["rig"], t["tp"], t["lut"], as64(t["F"]), T_o, 15,
                                     step_vox=STEP)
        say("headline temperature fit", t.get("iters", 0) + 15)
        with rte().Plan(t["g"], t["rig"], channels=1, step_vox=STEP) as p:
            Tg = dev(T_g)
            p.reconstruct_temperature(dev(t["F"]), Tg, 15)
            T_g = Tg.cpu().numpy()
        t.update(T_o=T_o, T_g=T_g, iters=t.get("iters", 0) + 15)
        e_o, _ = oracle.temp_map(t["tp"], t["lut"], T_o)
        e_g, _ = oracle.temp_map(t["tp"], t["lut"], as64(T_g))
        assert rel_rms(e_g[1], e_o[1]) <= VOLUME_RMS, t["iters"]
        vis = e_o[1] >= 1e-3 * e_o[1].max()
        assert vis.sum() > 1000
        assert np.sqrt(np.mean(((as64(T_g) - T_o)[vis] / 1400.0) ** 2)) <= VOLUME_RMS, t["iters"]


@pytest.mark.parametrize("upto", [15, 30])
def test_temperature_workload_fit_matches_oracle(upto):
    advance_temperature(upto)


def test_colour_hg_workload_inscatter_and_render_match_oracle():
    """The colour workload with Henyey-Greenstein in-scattering (g = 0.5, one
    in-scatter grid per view) at full size: every view's grid and the render
    of every view and channel within the render tolerance of the oracle."""
    c = colour()
    say("headline colour, Henyey-Greenstein g = 0.5")
    S_o = oracle.inscatter(c["g"], as64(c["em"]), as64(c["sig"]), s_res=M, n_dirs=DIRS, phase_g=0.5, rig=c["rig"])
    F_o = oracle.render(c["g"], c["rig"], as64(c["em"]), as64(c["sig"]), step_vox=STEP, albedo=ALBEDO,
                        inscatter=S_o)
    with rte().Plan(c["g"], c["rig"], channels=3, step_vox=STEP, albedo=ALBEDO, scatter_res=M,
                    scatter_dirs=DIRS, phase_g=0.5) as p:
        S = host(p.inscatter(dev(c["em"]), dev(c["sig"])))
        img = host(p.render(dev(c["em"]), dev(c["sig"]), dev(f32(S_o))))
    assert S.shape == S_o.shape == (VIEWS, 3, M, M, M)
    for v in range(VIEWS):
        assert np.abs(S[v] - S_o[v]).max() / np.abs(S_o[v]).max() <= RENDER_REL, v
    assert render_rel(img, F_o) <= RENDER_REL


def test_differentiable_workload_render_matches_oracle():
    """The differentiable workload's forward model at full size: 256^3 RGB
    emission + extinction from 20 plume blobs, single scattering (albedo 0.3,
    32^3 x 32 in-scatter grid), 12 views of 1024x768; the in-scatter grid and
    the render of every view and channel within the render tolerance."""
    g, em, sig = synth.colour_volume(0, n=256)
    rig = synth.ring_rig(12, 1024, 768)
    em, sig = f32(em), f32(sig)
    say("headline differentiable forward, 256^3 x 12 x 1024x768")
    S_o = oracle.inscatter(g, as64(em), as64(sig), s_res=M, n_dirs=DIRS)
    F_o = oracle.render(g, rig, as64(em), as64(sig), step_vox=STEP, albedo=ALBEDO, inscatter=S_o)
    with rte().Plan(g, rig, channels=3, step_vox=STEP, albedo=ALBEDO, scatter_res=M, scatter_dirs=DIRS,
                    gradients=True) as p:
        S = host(p.inscatter(dev(em), dev(sig)))
        img, _ = p.render_forward(dev(em), dev(sig), dev(f32(S_o)))
        img = host(img)
    assert np.abs(S - S_o).max() / np.abs(S_o).max() <= RENDER_REL
    assert render_rel(img, F_o) <= RENDER_REL
