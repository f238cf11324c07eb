"""The C boundary's stream semantics: a new observation is queued on a stream
behind the evaluations already queued there, with no device-wide wait, and
the tests run the in-tree library."""
import os

import numpy as np
import pytest
import torch

from paper_2606_30620_amd import synth
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def test_the_in_tree_library_is_loaded():
    from paper_2606_30620_amd import _lib
    here = os.path.dirname(os.path.abspath(_lib.__file__))
    assert os.path.samefile(_lib.LIB._name, os.path.join(here, "librtu.so"))


def test_observation_upload_is_ordered_on_its_stream():
    """Observation A, an evaluation, observation B (different mask size), an
    evaluation, all queued on one side stream without a host wait: each
    evaluation sees its own observation, bit for bit as a plan set up for that
    observation alone."""
    from paper_2606_30620_amd import api
    from paper_2606_30620_amd._lib import Plan, make_geometry
    g = synth.Geometry(96, 0.06, 2, 32, 15, 1.2)
    pa = synth.make_problem("X", batch=2, seed=51, geom=g)
    pb = synth.make_problem("X", batch=2, seed=52, geom=g)
    assert pa.mask.sum() != pb.mask.sum()
    say(f"[gpu] stream-ordered observations: masks of {int(pa.mask.sum())} and {int(pb.mask.sum())} pixels")
    geom = make_geometry(g.n_img, g.supersample, g.n_src, g.psf_size, g.pixel_scale)
    s = torch.cuda.Stream()
    plan = Plan(geom, 2)
    with torch.cuda.stream(s):
        la, psa, wa, na = api.device_inputs(pa)
        lb, psb, wb, nb = api.device_inputs(pb)
        plan.set_observation(pa.image, pa.noise_sigma, pa.psf, pa.mask, stream=s)
        ra = api.evaluate(plan, la, psa, wa, na, want_model=True, stream=s)
        plan.set_observation(pb.image, pb.noise_sigma, pb.psf, pb.mask, stream=s)
        rb = api.evaluate(plan, lb, psb, wb, nb, want_model=True, stream=s)
    s.synchronize()
    for p, r in ((pa, ra), (pb, rb)):
        ref_plan = api.plan_for_problem(p)
        l, ps_, w, n = api.device_inputs(p)
        ref = api.evaluate(ref_plan, l, ps_, w, n, want_model=True)
        torch.cuda.synchronize()
        for name in ("loss", "model", "grad_lens", "grad_ps", "grad_latent", "status"):
            assert torch.equal(getattr(r, name), getattr(ref, name)), name
