"""Randomised GPU parity (seeded, hypothesis-driven): small grids of any
shape (including fewer than 8 key points per axis), boxes off the unit cube,
1-3 cameras anywhere outside or inside the box with random orientation and
field of view, ragged images of 1-23 pixels per side, one or three channels.
Render, adjoint back-projection, in-scatter grids and render gradients through the C ABI against the FP64
oracle at every generated case; three iterations of reconstruction (SART, EM
or the paper's update; ordered subsets; in-scattering with or without the
phase function; flame mask and visual hull) likewise."""
import numpy as np
import pytest

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import HealthCheck, given, settings, strategies as st  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402
from gpu_util import BACKPROJ_REL, RENDER_REL, as64, dev, f32, host, rel_max, render_rel, say  # noqa: E402

pytestmark = pytest.mark.gpu


def rte():
    from paper_1809_06417_amd import rte as _rte
    return _rte


@st.composite
def cases(draw):
    nx, ny, nz = (draw(st.integers(2, 14)) for _ in range(3))
    lo = np.array([draw(st.floats(-1.0, 1.0)) for _ in range(3)])
    ext = np.array([draw(st.floats(0.3, 2.0)) for _ in range(3)])
    V = draw(st.integers(1, 3))
    W, H = draw(st.integers(1, 23)), draw(st.integers(1, 23))
    C = draw(st.sampled_from([1, 3]))
    seed = draw(st.integers(0, 2**31 - 1))
    inside = draw(st.booleans())
    return nx, ny, nz, lo, ext, V, W, H, C, seed, inside


def build(nx, ny, nz, lo, ext, V, W, H, C, seed, inside):
    rng = np.random.default_rng(seed)
    g = synth.Grid(nx, ny, nz, lo=tuple(lo), hi=tuple(lo + ext))
    centre = lo + ext / 2
    Rs, ts = [], []
    for v in range(V):
        if inside and v == 0:
            eye = lo + ext * rng.uniform(0.2, 0.8, 3)
        else:
            d = rng.normal(size=3)
            eye = centre + d / np.linalg.norm(d) * np.linalg.norm(ext) * rng.uniform(0.8, 3.0)
        target = centre + ext * rng.uniform(-0.3, 0.3, 3)
        up = np.array([0.0, 0.0, 1.0]) if abs((target - eye)[2]) < 0.9 * np.linalg.norm(target - eye) \
            else np.array([1.0, 0.0, 0.0])
        R, t = synth._look_at(eye, target, up)
        Rs.append(R)
        ts.append(t)
    fov = rng.uniform(20.0, 100.0)
    f = (H / 2.0) / np.tan(np.radians(fov) / 2.0)
    rig = synth.Rig(np.full(V, f), np.full(V, f * rng.uniform(0.8, 1.25)), np.full(V, W / 2.0),
                    np.full(V, H / 2.0), np.array(Rs), np.array(ts), W, H)
    em = f32(rng.uniform(0.0, 1.0, size=(C, nz, ny, nx)))
    sig = f32(rng.uniform(0.0, 3.0, size=(nz, ny, nx)) / np.min(ext))
    return g, rig, em, sig


@settings(max_examples=120, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(cases())
def test_random_render_and_backprojection_match_oracle(case):
    g, rig, em, sig = build(*case)
    C = em.shape[0]
    ref = oracle.render(g, rig, as64(em), as64(sig), step_vox=0.5, background=0.05)
    y = f32(np.random.default_rng(case[9] + 1).normal(size=ref.shape))
    bref = oracle.backproject_adjoint(g, rig, as64(sig), as64(y), step_vox=0.5)
    say("random case", case[:3], "views", case[5], "image", case[6:8], "C", C, "seed", case[9], "inside", case[10])
    with rte().Plan(g, rig, channels=C, step_vox=0.5, background=0.05) as p:
        img = host(p.render(dev(em), dev(sig)))
        d = host(p.backproject(dev(sig), dev(y)))
    assert render_rel(img, ref) <= RENDER_REL
    if np.abs(bref).max() > 0:
        assert rel_max(d, bref) <= BACKPROJ_REL
    else:
        assert np.abs(d).max() == 0.0


def random_case(rng, min_views=1):
    """A case of the same family as `cases`, drawn from a numpy generator."""
    nx, ny, nz = (int(n) for n in rng.integers(2, 15, 3))
    lo, ext = rng.uniform(-1.0, 1.0, 3), rng.uniform(0.3, 2.0, 3)
    V = int(rng.integers(min_views, 4))
    W, H = (int(n) for n in rng.integers(1, 24, 2))
    C = int(rng.choice([1, 3]))
    return nx, ny, nz, lo, ext, V, W, H, C, int(rng.integers(0, 2**31 - 1)), bool(rng.integers(0, 2))


# every combination of update rule, ordered subsets, in-scattering and
# restriction, each on its own random geometry
RECON_COMBOS = [(u, n, s, r) for u in ("sart", "mlem", "paper") for n in (1, 2)
                for s in ("none", "iso", "hg") for r in ("none", "mask", "hull")]


@pytest.mark.parametrize("combo", range(len(RECON_COMBOS)))
def test_random_reconstruction_matches_oracle(combo):
    update, subsets, scat, restrict = RECON_COMBOS[combo]
    rng = np.random.default_rng(1000 + combo)
    base = list(random_case(rng, min_views=subsets))
    if scat != "none":
        base[8] = 3
    g, rig, em, sig = build(*base)
    C = em.shape[0]
    scatter, phase_g = scat != "none", (0.6 if combo % 2 else -0.4) if scat == "hg" else 0.0
    masked, hull = restrict != "none", restrict == "hull"
    M = 4 if scatter else 0
    kw = dict(step_vox=0.5, albedo=0.3 if scatter else 0.0, background=0.0)
    S = oracle.inscatter(g, as64(em), as64(sig), s_res=4, n_dirs=8, phase_g=phase_g, rig=rig) if scatter else None
    F = f32(oracle.render(g, rig, as64(em), as64(sig), inscatter=S, **kw))
    thr = float(np.float32(0.05 * F.max())) if masked else None
    x0 = np.full(em.shape, 0.1)
    ref, _, _ = oracle.reconstruct_ext(g, rig, as64(F), as64(sig), x0, 3, s_res=4, n_dirs=8, phase_g=phase_g,
                                       mode=update, subsets=subsets, flame_threshold=thr, hull=hull,
                                       outside_value=0.0, **kw)
    say("random reconstruction", base[:3], "views", base[5], "image", base[6:8], "C", C, update, "subsets", subsets,
        "scatter", scat, phase_g, restrict, "seed", base[9])
    with rte().Plan(g, rig, channels=C, scatter_res=M, scatter_dirs=8, phase_g=phase_g, **kw) as p:
        x = host(p.reconstruct(dev(F), dev(sig), dev(x0), 3, update=update, subsets=subsets,
                               flame_threshold=thr, hull=hull))
    scale = np.abs(ref).max()
    if scale == 0:
        assert np.abs(x).max() == 0.0
        return
    same = np.ones(x.shape, dtype=bool)
    if hull:
        # key points on the hull boundary may be decided differently in FP32 and FP64
        inside_o = oracle.visual_hull(g, rig, oracle.flame_mask(as64(F), thr), step_vox=0.5)
        same = np.broadcast_to(inside_o, x.shape)
        if not same.any():
            return
    assert np.sqrt(np.mean((x - ref)[same] ** 2)) / scale <= 1e-3


@st.composite
def scatter_cases(draw):
    base = list(draw(cases()))
    base[8] = draw(st.sampled_from([1, 3]))
    M = draw(st.integers(2, 9))
    dirs = draw(st.integers(1, 24))
    g = draw(st.sampled_from([0.0, 0.0, 0.7, -0.5]))
    return base, M, dirs, g


@settings(max_examples=60, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(scatter_cases())
def test_random_inscatter_matches_oracle(sc):
    """In-scatter grids (isotropic and Henyey-Greenstein) on random grids and
    boxes, including face nodes of unevenly rounded boxes and directions that
    run along a face."""
    base, M, dirs, g = sc
    grid, rig, em, sig = build(*base)
    ref = oracle.inscatter(grid, as64(em), as64(sig), s_res=M, n_dirs=dirs, phase_g=g,
                           rig=rig if g != 0.0 else None)
    say("random in-scatter", base[:3], "C", base[8], "M", M, "dirs", dirs, "g", g, "seed", base[9])
    with rte().Plan(grid, rig, channels=base[8], step_vox=0.5, albedo=0.3, scatter_res=M, scatter_dirs=dirs,
                    phase_g=g) as p:
        S = host(p.inscatter(dev(em), dev(sig)))
    assert S.shape == ref.shape
    scale = np.abs(ref).max()
    if scale == 0.0:
        assert np.abs(S).max() == 0.0
    else:
        assert np.abs(S - ref).max() <= RENDER_REL * scale


@st.composite
def gradient_cases(draw):
    base = list(draw(cases()))
    scatter = draw(st.booleans())
    if scatter:
        base[8] = 3
    return base, scatter, draw(st.sampled_from([0.0, 0.6]))


@settings(max_examples=40, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(gradient_cases())
def test_random_render_gradient_matches_oracle(gc):
    """Gradients of a loss through the render (reverse march + gradient
    gather) on random geometry, with and without in-scattering."""
    base, scatter, g = gc
    grid, rig, em, sig = build(*base)
    C = em.shape[0]
    M = 4 if scatter else 0
    kw = dict(step_vox=0.5, albedo=0.3 if scatter else 0.0, background=0.05)
    S = oracle.inscatter(grid, as64(em), as64(sig), s_res=4, n_dirs=6, phase_g=g,
                         rig=rig if g != 0.0 else None) if scatter else None
    y = f32(np.random.default_rng(base[9] + 3).normal(size=(rig.n_views, C, rig.height, rig.width)))
    de_o, ds_o = oracle.render_grad(grid, rig, as64(em), as64(sig), as64(y), inscatter=S, **kw)
    say("random gradient", base[:3], "views", base[5], "image", base[6:8], "C", C, "scatter", scatter, g,
        "seed", base[9])
    with rte().Plan(grid, rig, channels=C, scatter_res=M, scatter_dirs=6, phase_g=g if scatter else 0.0,
                    gradients=True, **kw) as p:
        Sd = None if S is None else dev(f32(S))
        img, exit_tau = p.render_forward(dev(em), dev(sig), Sd)
        de, ds = p.render_backward(dev(em), dev(sig), Sd, exit_tau, dev(y))
        de, ds = host(de), host(ds)
    for got, ref in ((de, de_o), (ds, ds_o)):
        scale = np.abs(ref).max()
        if scale == 0.0:
            assert np.abs(got).max() == 0.0
        else:
            assert np.abs(got - ref).max() <= 1e-4 * scale
