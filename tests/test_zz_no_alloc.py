"""The allocation-free entry point (rtu_loss_grad_noalloc: no plan, every
intermediate in the library's static device array) against rtu_loss_grad on a
plan, through the C ABI: two calls in a row, the second on a smaller input
(smaller image, source grid, PSF and batch), each checked to the parity bar
(loss and images 1e-4, gradients 1e-3 relative to the group's largest value);
and a request larger than the array refused on the host."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2606_30620_amd import synth
from tests.gpu_helpers import TOL_GRAD, TOL_IMG, relinf, say

pytestmark = pytest.mark.gpu


def _noalloc(problem):
    from paper_2606_30620_amd import _lib, api
    g = problem.geom
    geom = _lib.make_geometry(g.n_img, g.supersample, g.n_src, g.psf_size, g.pixel_scale, g.n_sub_max,
                              g.tnfw_tau, 0, g.n_gauss)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    image, sigma, psf, mask = dev(problem.image), dev(problem.noise_sigma), dev(problem.psf), dev(problem.mask)
    lens, ps, lat, nsub = api.device_inputs(problem)
    B = problem.batch
    out = api.Result(loss=torch.empty(B, dtype=torch.float64, device="cuda"),
                     chi2_mask=torch.empty(B, dtype=torch.float64, device="cuda"),
                     status=torch.empty(B, dtype=torch.int32, device="cuda"),
                     grad_lens=torch.empty_like(lens), grad_ps=torch.empty_like(ps),
                     grad_latent=torch.empty_like(lat),
                     model=torch.empty((B, g.n_img, g.n_img), dtype=torch.float32, device="cuda"))
    p = lambda t: t.data_ptr()
    rc = _lib.LIB.rtu_loss_grad_noalloc(C.byref(geom), B, p(image), p(sigma), p(psf), p(mask), p(lens), p(nsub),
                                        p(ps), p(lat), p(out.loss), p(out.chi2_mask), p(out.grad_lens),
                                        p(out.grad_ps), p(out.grad_latent), p(out.model), p(out.status),
                                        torch.cuda.current_stream().cuda_stream)
    assert rc == 0, _lib.LIB.rtu_strerror(rc)
    return out


def _plan(problem):
    from paper_2606_30620_amd import api
    plan = api.plan_for_problem(problem)
    lens, ps, lat, nsub = api.device_inputs(problem)
    return plan, api.evaluate(plan, lens, ps, lat, nsub, want_model=True)


def test_noalloc_matches_plan_on_two_calls_the_second_smaller():
    big = synth.make_problem("X", batch=3, seed=61, geom=synth.Geometry(96, 0.06, 3, 64, 21, 1.2, n_sub_max=2,
                                                                         tnfw_tau=10.0, n_gauss=2))
    small = synth.make_problem("X", batch=2, seed=62, geom=synth.Geometry(48, 0.1, 2, 16, 9, 1.2))
    small.psf = np.ascontiguousarray(small.psf + 0.05 * small.psf.max() * np.eye(9, dtype=np.float32))  # rank > 1
    for name, prob in (("96x96 ss=3 n_src=64 psf=21, 2 subhaloes, 2 light, batch 3", big),
                       ("48x48 ss=2 n_src=16 psf=9 (rank two), batch 2", small)):
        say(f"[gpu] no-alloc vs plan: {name}")
        a = _noalloc(prob)
        plan, b = _plan(prob)
        torch.cuda.synchronize()
        assert torch.equal(a.status, b.status)
        for k in ("loss", "chi2_mask", "model"):
            assert relinf(getattr(a, k).cpu().numpy(), getattr(b, k).cpu().numpy()) <= TOL_IMG, k
        for k in ("grad_lens", "grad_ps", "grad_latent"):
            for s in range(prob.batch):
                assert relinf(getattr(a, k)[s].cpu().numpy(), getattr(b, k)[s].cpu().numpy()) <= TOL_GRAD, (k, s)
        same = all(torch.equal(getattr(a, k), getattr(b, k)) for k in
                   ("loss", "chi2_mask", "model", "grad_lens", "grad_ps", "grad_latent"))
        say(f"  bitwise equal to the plan's result: {same}")


def test_noalloc_refuses_more_than_the_static_array():
    from paper_2606_30620_amd import _lib
    g = synth.CONFIGS["C4"]
    geom = _lib.make_geometry(g.n_img, g.supersample, g.n_src, g.psf_size, g.pixel_scale)
    one = torch.zeros(16, device="cuda")
    p = one.data_ptr()
    rc = _lib.LIB.rtu_loss_grad_noalloc(C.byref(geom), 64, *([p] * 15), None)
    assert rc == _lib.RTU_ETOOBIG
