"""Parity of the weighted RTU grid (rtu_set_ray_weights, Sec. 6.3) on the GPU
with the oracle's weighted quantiles, and its contract: unit weights give the
unweighted grid bit for bit, NULL restores it, invalid weights are refused."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2606_30620_amd import synth
from tests.gpu_helpers import say
from tests.test_gpu_parity import _check, c1_mock

pytestmark = pytest.mark.gpu


def _brightness_weights(p, floor=0.2):
    img = np.abs(p.image.astype(np.float64))
    w = img / img[p.mask.astype(bool)].mean()
    w[w < floor] = 0.0
    return w.astype(np.float32)


def test_weighted_c2_batch():
    say("[gpu] weighted RTU grid: C2 200x200 ss=4 n_src=64, brightness weights, batch 3")
    p = synth.make_problem("C2", batch=3)
    p = dataclasses.replace(p, ray_weights=_brightness_weights(p))
    _check(p, range(3))


def test_weighted_c1_and_integer_weights():
    say("[gpu] weighted RTU grid: C1 with brightness weights; C1 with integer weights 1..3")
    p = c1_mock()
    _check(dataclasses.replace(p, ray_weights=_brightness_weights(p)), [0])
    w = np.random.default_rng(3).integers(1, 4, p.mask.shape).astype(np.float32)
    _check(dataclasses.replace(p, ray_weights=w), [0])


def test_unit_weights_are_bitwise_unweighted_and_none_restores():
    from paper_2606_30620_amd import _lib, api
    p = synth.make_problem("C2", batch=2)
    plan = api.plan_for_problem(p)
    lens, ps, lat, nsub = api.device_inputs(p)
    a = api.evaluate(plan, lens, ps, lat, nsub)
    plan.set_ray_weights(np.ones(p.mask.shape, np.float32))
    b = api.evaluate(plan, lens, ps, lat, nsub)
    plan.set_ray_weights(_brightness_weights(p))
    c = api.evaluate(plan, lens, ps, lat, nsub)
    plan.set_ray_weights(None)
    d = api.evaluate(plan, lens, ps, lat, nsub)
    torch.cuda.synchronize()
    for x in (b, d):
        assert torch.equal(a.loss, x.loss) and torch.equal(a.grad_lens, x.grad_lens)
        assert torch.equal(a.grad_latent, x.grad_latent)
    assert not torch.equal(a.loss, c.loss)
    with pytest.raises(_lib.RTUError):
        plan.set_ray_weights(-np.ones(p.mask.shape, np.float32))
    with pytest.raises(_lib.RTUError):
        plan.set_ray_weights(np.full(p.mask.shape, 1e-6, np.float32))     # total weight below 1
