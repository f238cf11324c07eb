"""Parity of the elliptical power law deflector (RTU_GEOM_EPL, App. A.1,
eq. A1) on the GPU with the oracle's EPL: loss, images and gradients
(slope included) to the tolerances of the SIE parity tests; at slope 2 the
two deflectors agree; an ELBO + Adam step with the slope in the guide."""
import numpy as np
import pytest
import torch

from paper_2606_30620_amd import synth
from tests.gpu_helpers import say
from tests.test_gpu_parity import _check, c1_mock

pytestmark = pytest.mark.gpu


def test_epl_c1():
    say("[gpu] EPL: C1 64x64 ss=1 n_src=32, slope 2.1")
    _check(synth.with_epl(c1_mock()), [0])


def test_epl_c2_batch():
    say("[gpu] EPL: C2 200x200 ss=4 n_src=64, batch 3, slopes around 2.2")
    _check(synth.with_epl(synth.make_problem("C2", batch=3), slope_mean=2.2, slope_spread=0.1), range(3))


def test_epl_subhaloes_light_and_global_grid():
    say("[gpu] EPL: 80x80 ss=2 n_src=128 with 2 subhaloes; 48x48 with 3 lens-light Gaussians; slopes 1.8-2.4")
    g = synth.Geometry(80, 0.06, 2, 128, 21, 0.85, n_sub_max=2, tnfw_tau=10.0)
    _check(synth.with_epl(synth.make_problem("X", batch=2, seed=9, geom=g), slope_mean=1.85), range(2))
    g = synth.Geometry(48, 0.08, 2, 16, 15, 1.0, n_gauss=3)
    _check(synth.with_epl(synth.make_problem("X", batch=2, seed=31, geom=g), slope_mean=2.4), range(2))


def test_epl_at_slope_two_is_the_sie():
    from paper_2606_30620_amd import api
    p = synth.make_problem("C2", batch=2)
    q = synth.with_epl(p, slope_mean=2.0, slope_spread=0.0)
    out = []
    for prob in (p, q):
        plan = api.plan_for_problem(prob)
        lens, ps, lat, nsub = api.device_inputs(prob)
        out.append(api.evaluate(plan, lens, ps, lat, nsub))
    torch.cuda.synchronize()
    a, b = out
    assert torch.allclose(a.loss, b.loss, rtol=2e-5)
    ga, gb = a.grad_lens.cpu().numpy(), b.grad_lens.cpu().numpy()[:, :7]
    assert np.abs(ga - gb).max() <= 2e-3 * np.abs(ga).max()
    assert torch.allclose(a.grad_latent, b.grad_latent, rtol=1e-3, atol=1e-3 * float(a.grad_latent.abs().max()))


def test_elbo_step_with_epl_slope_matches_oracle():
    from tests.test_gpu_fit import _elbo_step_check
    say("[gpu] fit: one ELBO+Adam step with the EPL slope in the guide, 48x48 ss=2 n_src=16, S=2")
    g = synth.Geometry(48, 0.08, 2, 16, 15, 1.0)
    p = synth.with_epl(synth.make_problem("X", batch=1, seed=35, geom=g))
    _elbo_step_check(p, {"lens": slice(0, 8), "ps": slice(8, 12), "latent": slice(12, None)})
