"""GPU parity of ordered-subset updates (per-view SART, OS-EM, paper mode by
subsets): views v mod n form subset v % n, one update per subset with the
subset's own row and column sums, against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import VOLUME_RMS, as64, dev, host, rel_rms, say
from test_gpu_parity import STEP, case, oracle_frames
from test_gpu_variants import flame_case

pytestmark = pytest.mark.gpu


def rte():
    from paper_1809_06417_amd import rte as _rte
    return _rte


@pytest.mark.parametrize("update,n", [("sart", 2), ("sart", 4), ("mlem", 2), ("paper", 4)])
def test_ordered_subsets_colour_with_inscatter(update, n):
    c = case("colour_small")
    F = oracle_frames(c)
    x0 = np.full(c["em"].shape, 0.02)
    ref, _, it = oracle.reconstruct_ext(c["g"], c["rig"], as64(F), as64(c["sig"]), x0, 3, step_vox=STEP,
                                        albedo=c["albedo"], background=c["bg"], s_res=c["M"], n_dirs=c["dirs"],
                                        mode=update, subsets=n)
    assert it == 3
    say("ordered subsets", update, n)
    with rte().Plan(c["g"], c["rig"], channels=3, step_vox=STEP, albedo=c["albedo"], background=c["bg"],
                    scatter_res=c["M"], scatter_dirs=c["dirs"]) as p:
        x = host(p.reconstruct(dev(F), dev(c["sig"]), dev(x0), 3, update=update, subsets=n))
        assert p.stats()[0] == 3
    for ch in range(3):
        assert rel_rms(x[ch], ref[ch]) <= VOLUME_RMS


def test_per_view_sart_with_mask_and_hull():
    g, rig, em, sig, F, thr = flame_case()
    n = rig.n_views
    ref, _, _ = oracle.reconstruct_ext(g, rig, as64(F), as64(sig), np.zeros(em.shape), 3, step_vox=STEP,
                                       flame_threshold=thr, hull=True, outside_value=-1e-3, subsets=n)
    say("per-view SART, mask + hull")
    with rte().Plan(g, rig, channels=1, step_vox=STEP) as p:
        x = host(p.reconstruct(dev(F), dev(sig), dev(np.zeros(em.shape)), 3, flame_threshold=thr, hull=True,
                               outside_value=-1e-3, subsets=n))
        inside = p.visual_hull(p.flame_mask(dev(F), thr)).cpu().numpy().astype(bool)
    ref_in = oracle.visual_hull(g, rig, oracle.flame_mask(as64(F), thr), step_vox=STEP)
    same = inside == ref_in
    assert np.all(x[0][~inside] == np.float32(-1e-3))
    assert rel_rms(x[0][same], ref[0][same]) <= VOLUME_RMS


def test_one_subset_is_the_simultaneous_update():
    import torch
    c = case("tiny")
    F = oracle_frames(c)
    say("one subset")
    with rte().Plan(c["g"], c["rig"], channels=1, step_vox=STEP) as p:
        a = p.reconstruct(dev(F), dev(c["sig"]), dev(np.zeros(c["em"].shape)), 3, subsets=1)
        b = p.reconstruct(dev(F), dev(c["sig"]), dev(np.zeros(c["em"].shape)), 3, subsets=0)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


def test_ordered_subsets_reject_unsupported_combinations():
    c = case("tiny")
    F = oracle_frames(c)
    say("subset errors")
    with rte().Plan(c["g"], c["rig"], channels=1, step_vox=STEP) as p:
        x = dev(np.zeros(c["em"].shape))
        for kw in (dict(subsets=c["rig"].n_views + 1), dict(subsets=2, stop_tol=1e-3),
                   dict(subsets=2, update="paper", g_sigma=0.5)):
            with pytest.raises(rte().RteError):
                p.reconstruct(dev(F), dev(c["sig"]), x, 2, **kw)
        assert float(x.abs().max()) == 0.0  # rejected before any work
