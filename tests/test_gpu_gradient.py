"""GPU parity of the differentiable render: the reverse-march adjoint against
the FP64 oracle gradient, the autograd wrapper, and central finite
differences at the full differentiation workload."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import as64, dev, f32, host, rel_max, say
from test_gpu_parity import STEP, case, oracle_S

pytestmark = pytest.mark.gpu

GRAD_REL = 1e-4  # max |grad_gpu - grad_orc| / max |grad_orc|, per field


def rte():
    from paper_1809_06417_amd import rte as _rte
    return _rte


@pytest.mark.parametrize("name", ["tiny", "ragged", "colour_small"])
def test_render_gradient_matches_oracle(name):
    c = case(name)
    S = oracle_S(c)
    rng = np.random.default_rng(6)
    sig = f32(as64(c["sig"]) + 0.05)  # strictly positive extinction: no kink of max(0, .)
    F = f32(rng.uniform(0.0, 0.2, size=(c["rig"].n_views, c["C"], c["rig"].height, c["rig"].width)))
    kw = dict(step_vox=STEP, albedo=c["albedo"], background=c["bg"],
              inscatter=None if S is None else as64(S))
    I = oracle.render(c["g"], c["rig"], as64(c["em"]), as64(sig), **kw)
    y = f32(I - as64(F))
    de_o, ds_o = oracle.render_grad(c["g"], c["rig"], as64(c["em"]), as64(sig), as64(y), **kw)
    say("render gradient", name)
    with rte().Plan(c["g"], c["rig"], channels=c["C"], step_vox=STEP, albedo=c["albedo"],
                    background=c["bg"], scatter_res=c.get("M", 0), scatter_dirs=c.get("dirs", 32),
                    gradients=True) as p:
        Sd = None if S is None else dev(S)
        img, exit_T = p.render_forward(dev(c["em"]), dev(sig), Sd)
        de, ds = p.render_backward(dev(c["em"]), dev(sig), Sd, exit_T, dev(y))
        de, ds = host(de), host(ds)
    assert rel_max(de, de_o) <= GRAD_REL
    assert rel_max(ds, ds_o) <= GRAD_REL


def test_autograd_function_matches_backward_and_finite_differences():
    import torch
    from paper_1809_06417_amd import autograd
    c = case("colour_small")
    S = dev(oracle_S(c))
    F = dev(np.random.default_rng(7).uniform(0.0, 0.2, size=(4, 3, 36, 40)))
    say("autograd")
    with rte().Plan(c["g"], c["rig"], channels=3, step_vox=STEP, albedo=c["albedo"], background=c["bg"],
                    scatter_res=c["M"], scatter_dirs=c["dirs"], gradients=True) as p:
        em = dev(c["em"]).requires_grad_(True)
        sig = dev(as64(c["sig"]) + 0.05).requires_grad_(True)
        loss = 0.5 * ((autograd.render(p, em, sig, S) - F) ** 2).sum()
        loss.backward()
        with torch.no_grad():
            img, exit_T = p.render_forward(em.detach(), sig.detach(), S)
            de, ds = p.render_backward(em.detach(), sig.detach(), S, exit_T, (img - F).contiguous())
        assert torch.equal(em.grad, de) and torch.equal(sig.grad, ds)

        def L(e, s):
            with torch.no_grad():
                return 0.5 * ((p.render(e, s, S) - F).double() ** 2).sum().item()
        rng = np.random.default_rng(3)
        for _ in range(6):
            ch, z, yy, x = rng.integers(0, 3), *rng.integers(6, 18, size=3)
            for field, grad in ((em, em.grad), (sig, sig.grad)):
                idx = (ch, z, yy, x) if field is em else (z, yy, x)
                base = field.detach().clone()
                plus, minus = base.clone(), base.clone()
                plus[idx] += 1e-3
                minus[idx] -= 1e-3
                dx = (plus[idx] - minus[idx]).item()
                a = (L(plus, sig.detach()) - L(minus, sig.detach())) / dx if field is em else \
                    (L(em.detach(), plus) - L(em.detach(), minus)) / dx
                g = grad[idx].item()
                assert abs(a - g) <= 2e-2 * max(abs(g), 1e-4), (idx, a, g)


def test_full_size_gradient_against_finite_differences():
    """The differentiation workload: 256^3 RGB emission + extinction with single
    scattering, 12 views of 1024x768; L2 image loss; central differences with
    h = 1e-3 on 64 random voxels inside the flame."""
    import torch
    g, em_gt, sig_gt = synth.colour_volume(seed=4, n=256)
    rig = synth.ring_rig(12, 1024, 768)
    say("full-size gradient FD")
    with rte().Plan(g, rig, channels=3, step_vox=STEP, albedo=0.3, scatter_res=32, scatter_dirs=32,
                    gradients=True) as p:
        emg, sgg = dev(em_gt), dev(sig_gt)
        S = p.inscatter(emg, sgg)
        F = p.render(emg, sgg, S)
        em = (emg * 0.8).contiguous()
        sig = (sgg * 0.9 + 0.02).contiguous()
        img, exit_T = p.render_forward(em, sig, S)
        de, ds = p.render_backward(em, sig, S, exit_T, (img - F).contiguous())

        def L(e, s):
            return 0.5 * ((p.render(e, s, S) - F).double() ** 2).sum().item()
        rng = np.random.default_rng(11)
        inside = np.argwhere(sig_gt > 0.5)
        picks = inside[rng.choice(len(inside), size=64, replace=False)]
        errs = []
        for i, (z, yy, x) in enumerate(picks):
            if i % 2 == 0:
                ch = int(rng.integers(0, 3))
                base, idx, grad = em, (ch, z, yy, x), de
            else:
                base, idx, grad = sig, (z, yy, x), ds
            plus, minus = base.clone(), base.clone()
            plus[idx] += 1e-3
            minus[idx] -= 1e-3
            dx = (plus[idx] - minus[idx]).item()
            if base is em:
                fd = (L(plus, sig) - L(minus, sig)) / dx
            else:
                fd = (L(em, plus) - L(em, minus)) / dx
            gval = grad[idx].item()
            errs.append(abs(fd - gval) / max(abs(gval), 1e-3 * float(grad.abs().max())))
    errs = np.array(errs)
    assert np.median(errs) <= 5e-3 and errs.max() <= 3e-2, errs


def test_adam_reconstruction_reduces_loss():
    import torch
    from paper_1809_06417_amd import autograd
    c = case("colour_small")
    S = dev(oracle_S(c))
    say("adam")
    with rte().Plan(c["g"], c["rig"], channels=3, step_vox=STEP, albedo=c["albedo"], background=c["bg"],
                    scatter_res=c["M"], scatter_dirs=c["dirs"], gradients=True) as p:
        F = p.render(dev(c["em"]), dev(c["sig"]), S)
        em = torch.full((3,) + c["g"].shape_zyx, 0.1, device="cuda", requires_grad=True)
        sig = torch.full(c["g"].shape_zyx, 0.5, device="cuda", requires_grad=True)
        opt = torch.optim.Adam([em, sig], lr=0.05)
        losses = []
        for _ in range(50):
            opt.zero_grad()
            loss = 0.5 * ((autograd.render(p, em, sig, S) - F) ** 2).sum()
            loss.backward()
            opt.step()
            with torch.no_grad():
                em.clamp_(min=0)
                sig.clamp_(min=0)
            losses.append(loss.item())
    assert losses[-1] < 0.1 * losses[0]
