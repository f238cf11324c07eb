"""GPU parity at the lens model's degenerate points (App. A.1): a round lens
(e1 = e2 = 0, where the position angle is undefined and the gradient with
respect to (e1, e2) is formed without it), ellipticities on both sides of the
switch between the two forms of that gradient, and a sub-ray exactly on the
lens centre (not deflected).  Then the GPU gradient with respect to the latent
and the spectrum parameters against central differences of the GPU loss at C2
(h = 1e-4).  Tolerances as in tests/gpu_helpers.py."""
import numpy as np
import pytest
import torch

from paper_2606_30620_amd import synth
from tests.gpu_helpers import say
from tests.test_gpu_parity import _check

pytestmark = pytest.mark.gpu


def test_round_lens_and_both_sides_of_the_gradient_switch():
    g = synth.Geometry(64, 0.09, 2, 32, 15, 1.2)
    p = synth.make_problem("X", batch=4, seed=31, geom=g)
    lens = p.lens.astype(np.float64)
    for b, e in enumerate((0.0, 0.01, 0.0199, 0.0201)):
        ang = 0.4 + b
        lens[b, 1], lens[b, 2] = e * np.cos(ang), e * np.sin(ang)
    p.lens = lens.astype(np.float32)
    say("[gpu] round lens (e = 0) and e = 0.01, 0.0199, 0.0201: 64x64 ss=2 n_src=32 psf=15, batch 4")
    _, res, _ = _check(p, range(4))
    assert bool(torch.isfinite(res.grad_lens).all())


def test_subray_on_the_lens_centre():
    """The lens centre sits exactly on sub-ray (0, 0) of pixel (N/2, N/2):
    (1/4, 1/4) of a pixel, exact in binary32 and binary64, so both sides put
    that ray at psi = 0.  Sample 1 is also a round lens."""
    g = synth.Geometry(64, 0.09, 2, 32, 15, 1.2)
    p = synth.make_problem("X", batch=2, seed=37, geom=g)
    c = 0.25 * float(np.float32(g.pixel_scale))
    lens = p.lens.copy()
    lens[:, 3] = np.float32(c)
    lens[:, 4] = np.float32(c)
    lens[1, 1] = lens[1, 2] = 0.0
    p.lens = lens
    assert float(np.float32(c)) == c
    say("[gpu] sub-ray on the lens centre: 64x64 ss=2 n_src=32 psf=15, batch 2 (sample 1 round)")
    _, res, _ = _check(p, range(2))
    assert int(res.status[0]) == 0 and int(res.status[1]) == 0


def test_gradient_matches_central_differences_of_the_gpu_loss():
    """C2 geometry, 2 samples: the library's gradient with respect to the
    spectrum parameters (sigma, n, zeta, alpha) and the latent w against
    central differences of the library's own loss.  The grid does not depend on
    w or the spectrum, so the loss is smooth there.  The latent moves along
    v = unit(g/|g| + r), r a random unit direction.  Each input step is the FP32
    difference actually taken, so the first-order prediction is
    sum_i g_i (x+ - x-)_i.

    Step: h = 1e-4 where that changes the loss by at least 20, else the step
    that does (at most 5 % of the parameter).  The loss, an FP64 sum of FP32
    pixel terms of about 2e4 at C2, carries rounding noise of 1e-2 to 3e-2
    (measured: central differences of a change of 10 missed by up to 0.03,
    depending on how the compiler orders the forward's FP32 arithmetic), so a
    change of 20 resolves the derivative to about 1e-3; the truncation error
    of the larger steps is O(h^2), below that."""
    from paper_2606_30620_amd import api
    p = synth.make_problem("C2", batch=2)
    plan = api.plan_for_problem(p)
    lens, ps, lat, nsub = api.device_inputs(p)
    base = api.evaluate(plan, lens, ps, lat, nsub)
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    worst = 0.0
    for d in range(5):
        if d < 4:
            what = ("sigma", "n", "zeta", "alpha")[d]
            e = torch.zeros_like(ps)
            e[:, d] = 1.0
            gdir = (base.grad_ps.double() * e.double()).sum(dim=1)
            scale = ps[:, d].abs().double()
        else:
            what = "w"
            g = base.grad_latent.double()
            r = torch.from_numpy(rng.standard_normal(lat.shape)).cuda()
            v = g / g.norm(dim=(1, 2), keepdim=True) + r / r.norm(dim=(1, 2), keepdim=True)
            e = (v / v.norm(dim=(1, 2), keepdim=True)).float()
            gdir = (g * e.double()).sum(dim=(1, 2))
            scale = torch.ones_like(gdir)
        h = torch.clamp(torch.maximum(torch.full_like(gdir, 1e-4), 20.0 / gdir.abs()), max=0.05 * scale).float()
        hb = h.view(-1, *([1] * (e.dim() - 1)))
        xp_, xm_ = ((ps + hb * e, ps - hb * e) if d < 4 else (lat + hb * e, lat - hb * e))
        if d < 4:
            pred = (base.grad_ps.double() * (xp_ - xm_).double()).sum(dim=1)
            lp = api.evaluate(plan, lens, xp_, lat, nsub, want_grad=False).loss
            lm = api.evaluate(plan, lens, xm_, lat, nsub, want_grad=False).loss
        else:
            pred = (base.grad_latent.double() * (xp_ - xm_).double()).sum(dim=(1, 2))
            lp = api.evaluate(plan, lens, ps, xp_, nsub, want_grad=False).loss
            lm = api.evaluate(plan, lens, ps, xm_, nsub, want_grad=False).loss
        torch.cuda.synchronize()
        fd = lp - lm
        rel = ((fd - pred).abs() / pred.abs().clamp_min(1e-30)).max().item()
        say(f"  d/d {what}: h {h.cpu().numpy()}, predicted change {pred.cpu().numpy()}, "
            f"central difference {fd.cpu().numpy()}, rel {rel:.2e}")
        worst = max(worst, rel)
        assert rel < 2e-3, (what, rel)
    say(f"  worst relative difference {worst:.2e}")
