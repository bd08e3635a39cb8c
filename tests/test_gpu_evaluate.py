"""GPU runs of the paper's evaluation protocols (Sec. 5) against the same
protocols carried out with the FP64 oracle: leave-one-view-out (input and
held-out view errors, volume error in the hull) and the camera-count sweep
of the temperature reconstruction (errors fall as cameras are added)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import as64, dev, f32, say
from test_gpu_parity import STEP, case

pytestmark = pytest.mark.gpu


def rmse_box(I, F, thr, scale):
    """Per view and channel RMSE inside the flame rectangle (written out
    separately from the library's evaluation helpers)."""
    V, C = F.shape[:2]
    out = np.zeros((V, C))
    for v in range(V):
        hot = np.argwhere((F[v] > thr).any(axis=0))
        (v0, u0), (v1, u1) = hot.min(axis=0), hot.max(axis=0) + 1
        out[v] = np.sqrt(((I[v, :, v0:v1, u0:u1] - F[v, :, v0:v1, u0:u1]) ** 2).mean(axis=(1, 2))) * scale
    return out


def test_leave_one_view_out_matches_oracle_protocol():
    from paper_1809_06417_amd import evaluate
    c = case("colour_small")
    g, rig, em, sig = c["g"], c["rig"], c["em"], c["sig"]
    kw = dict(step_vox=STEP, albedo=c["albedo"], background=c["bg"])
    say("leave one view out")
    got = evaluate.leave_one_view_out(g, rig, dev(em), dev(sig), 2, 4, scatter_res=c["M"],
                                      scatter_dirs=c["dirs"], **kw)
    # the same protocol with the oracle
    S = oracle.inscatter(g, as64(em), as64(sig), s_res=c["M"], n_dirs=c["dirs"])
    F = f32(oracle.render(g, rig, as64(em), as64(sig), inscatter=S, **kw))
    inputs = [0, 1, 3]
    x = oracle.reconstruct(g, rig.subset(inputs), as64(F[inputs]), as64(sig), np.zeros(em.shape), 4,
                           s_res=c["M"], n_dirs=c["dirs"], **kw)
    I = oracle.render(g, rig, x, as64(sig), inscatter=oracle.inscatter(g, x, as64(sig), s_res=c["M"],
                                                                        n_dirs=c["dirs"]), **kw)
    thr = 0.01 * F.max()
    err = rmse_box(I, as64(F), thr, 255.0 / F.max())
    inside = oracle.visual_hull(g, rig.subset(inputs), oracle.flame_mask(F[inputs], thr))
    vol = np.sqrt(((x - as64(em))[:, inside] ** 2).mean(axis=1)) * 255.0 / em.max()
    np.testing.assert_allclose(got["input"], err[inputs].mean(axis=0), rtol=0, atol=0.3)
    np.testing.assert_allclose(got["test"], err[2], rtol=0, atol=0.3)
    np.testing.assert_allclose(got["volume"], vol, rtol=0, atol=0.5)
    assert np.all(got["test"] > 0)


def test_camera_sweep_matches_oracle_and_errors_fall_with_cameras():
    import torch
    from paper_1809_06417_amd import evaluate
    g, T = synth.temperature_volume(0, n=24)
    T = f32(T)
    rigs = [synth.ring_rig(n, 48, 48, elevation_jitter_deg=10, seed=0) for n in (2, 4, 8)]
    say("camera sweep")
    got = evaluate.camera_sweep(g, torch.tensor(T, device="cuda"), rigs, 20)
    tp = oracle.TempParams()
    lut = oracle.temp_lut(tp)
    em3, sg = oracle.temp_map(tp, lut, as64(T))
    for rig, r in zip(rigs, got):
        F = np.stack([oracle.render(g, rig, em3[c:c + 1], sg, step_vox=STEP)[:, 0] for c in range(3)], 1)
        Tr = oracle.temperature_fit(g, rig, tp, lut, F, np.full(T.shape, 800.0), 20, step_vox=STEP)
        inside = oracle.visual_hull(g, rig, oracle.flame_mask(F[:, 1:2], 0.01 * F.max()))
        m = inside & (em3[1] >= 1e-3 * em3[1].max())
        t_rmse = np.sqrt(((Tr - as64(T))[m] ** 2).mean())
        assert abs(r["temperature_K"] - t_rmse) <= 0.03 * t_rmse, (rig.n_views, r["temperature_K"], t_rmse)
        assert abs(r["voxels"] - int(m.sum())) <= 0.01 * m.sum()
    t = [r["temperature_K"] for r in got]
    assert t[0] > t[1] > t[2]
