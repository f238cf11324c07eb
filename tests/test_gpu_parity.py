"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: images and loss within 1e-4 of the reference's infinity norm,
gradients within 1e-3 per parameter group.  Where an order statistic of the
masked rays is a near-tie, FP32 and FP64 may pick different (equally valid)
rays; then the pick is checked to be a valid alternative and the lens
gradient, which depends on which ray was picked, is compared with the
oracle's gradient for the GPU's picks (tests/gpu_helpers.py)."""
import math

import numpy as np
import pytest
import torch

from oracle import rtu_oracle as O
from paper_2606_30620_amd import _lib, synth
from tests.gpu_helpers import compare, say

pytestmark = pytest.mark.gpu


def _run(problem, samples=None, want_grad=True, batch_max=None, flags=0):
    from paper_2606_30620_amd import api
    plan = api.plan_for_problem(problem, max_batch=batch_max, flags=flags)
    lens, ps, lat, nsub = api.device_inputs(problem)
    res = api.evaluate(plan, lens, ps, lat, nsub, want_grad=want_grad, want_model=True)
    torch.cuda.synchronize()
    return plan, res


def _check(problem, samples, want_grad=True, check_stages=True, flags=0):
    plan, res = _run(problem, want_grad=want_grad, flags=flags)
    worst = {}
    for b in samples:
        ref = O.loss_grad_problem(problem, b, want_grad=want_grad, return_all=True)
        out = compare(plan, problem, b, res, ref, check_stages=check_stages)
        say(f"  sample {b}: " + ", ".join(f"{k}={v:.2e}" if isinstance(v, float) else f"{k}={v}"
                                          for k, v in out.items()))
        for k, v in out.items():
            if isinstance(v, float):
                worst[k] = max(worst.get(k, 0.0), v)
    return plan, res, worst


def c1_mock():
    """C1 with the observed image = oracle model at the truth + seeded noise."""
    p = synth.make_problem("C1")
    r = O.loss_grad_problem(p, 0, want_grad=False)
    p.image = (r["model"].detach().numpy() + p.noise.astype(np.float64)).astype(np.float32)
    # evaluate away from the truth so gradients are not near zero
    p.lens[0] = (p.lens[0].astype(np.float64) + np.array([0.01, 0.005, -0.004, 0.003, -0.002, 0.001, 0.002])
                 ).astype(np.float32)
    return p


def test_c1_full_parity():
    say("[gpu] C1 64x64 ss=1 n_src=32 psf=15, 1 sample")
    _check(c1_mock(), [0])


def test_c2_full_size_parity():
    say("[gpu] C2 200x200 ss=4 n_src=64 psf=21, batch 4 (all compared)")
    p = synth.make_problem("C2", batch=4)
    _check(p, range(4))


def test_ragged_generic_psf_parity():
    say("[gpu] ragged 72x72 ss=3 n_src=16 psf=9 (generic PSF kernel), batch 3")
    g = synth.Geometry(72, 0.06, 3, 16, 9, 1.2)
    p = synth.make_problem("X", batch=3, seed=7, geom=g)
    _check(p, range(3))


def _rank_two_psf(psf):
    """The problem's (Gaussian, rank-one) PSF plus a shifted, elongated lobe:
    rank two, so the matrix-core PSF kernel runs instead of the separable one."""
    K = psf.shape[0]
    a = np.arange(K) - K // 2
    lobe = np.exp(-0.5 * ((a[:, None] - 2.0) ** 2 / 2.0 + (a[None, :] + 1.0) ** 2 / 0.7))
    w = psf.astype(np.float64) + 0.2 * psf.max() * lobe / lobe.max()
    return (w / w.sum()).astype(np.float32)


@pytest.mark.parametrize("psf_size", [21, 9])
def test_rank_two_psf_parity(psf_size):
    say(f"[gpu] PSF of rank two ({psf_size}x{psf_size}, matrix-core PSF kernel): 96x96 ss=2 n_src=32, batch 2")
    g = synth.Geometry(96, 0.05, 2, 32, psf_size, 1.4)
    p = synth.make_problem("X", batch=2, seed=13, geom=g)
    p.psf = _rank_two_psf(p.psf)
    assert np.linalg.matrix_rank(p.psf.astype(np.float64), tol=1e-4 * np.abs(p.psf).max()) == 2
    _check(p, range(2))


def test_smallest_source_grid_parity():
    say("[gpu] n_src=8 (one 8-point FFT factor per line): 48x48 ss=2 psf=15, batch 2")
    g = synth.Geometry(48, 0.08, 2, 8, 15, 1.2)
    p = synth.make_problem("X", batch=2, seed=11, geom=g)
    _check(p, range(2))


def test_subhalo_parity():
    say("[gpu] subhaloes: 96x96 ss=2 n_src=64 psf=15, 3 truncated NFW, batch 2")
    g = synth.Geometry(96, 0.05, 2, 64, 15, 1.0, n_sub_max=3, tnfw_tau=10.0)
    p = synth.make_problem("X", batch=2, seed=11, geom=g)
    _check(p, range(2))


@pytest.mark.parametrize("n_sub_max, n_gauss", [(0, 5), (2, 3)])
def test_lens_light_parity(n_sub_max, n_gauss):
    say(f"[gpu] lens light: 80x80 ss=3 n_src=32 psf=15, {n_gauss} Gaussians, {n_sub_max} subhalo slots, batch 2")
    g = synth.Geometry(80, 0.06, 3, 32, 15, 1.0, n_sub_max=n_sub_max, tnfw_tau=10.0 if n_sub_max else 0.0,
                       n_gauss=n_gauss)
    p = synth.make_problem("X", batch=2, seed=23, geom=g)
    _check(p, range(2))


def test_lens_light_narrow_component_parity():
    """A lens-light component much narrower than the sub-ray spacing (sigma =
    0.004 arcsec against 0.02) makes the row recurrence's factors leave the
    FP32 range; those rows take one exponential per sub-ray and the result
    stays finite and equal to the oracle's."""
    say("[gpu] lens light with a 0.004 arcsec component: 64x64 ss=3 n_src=32 psf=15, batch 2")
    g = synth.Geometry(64, 0.06, 3, 32, 15, 1.0, n_gauss=2)
    p = synth.make_problem("X", batch=2, seed=41, geom=g)
    lens = p.lens.astype(np.float64)
    lens[:, 7 + 6 + 1] = 0.004              # second component's sigma
    lens[:, 7 + 6 + 4] = 0.3                # its centre, so that pixels lie on both sides
    p.lens = lens.astype(np.float32)
    _check(p, range(2))


def test_misaligned_latent_is_rejected():
    """The latent is read four floats at a time: a pointer that is not 16-byte
    aligned is refused on the host (RTU_EINVAL) before anything is launched."""
    say("[gpu] misaligned latent pointer -> RTU_EINVAL")
    from paper_2606_30620_amd import _lib, api
    p = synth.make_problem("C1")
    plan = api.plan_for_problem(p)
    lens, ps, lat, nsub = api.device_inputs(p)
    buf = torch.zeros(lat.numel() + 4, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    status = torch.empty(1, dtype=torch.int32, device="cuda")
    L = _lib.LIB
    vp = lambda t: t.data_ptr()
    rc = L.rtu_loss_grad(plan._h, 1, vp(lens), None, vp(ps), buf.data_ptr() + 4, vp(loss), None, None, None,
                         None, None, vp(status), None)
    assert rc == _lib.RTU_EINVAL
    rc = L.rtu_loss_grad(plan._h, 1, vp(lens), None, vp(ps), buf.data_ptr(), vp(loss), None, None, None,
                         None, None, vp(status), None)
    torch.cuda.synchronize()
    assert rc == 0


def test_large_source_grid_parity():
    say("[gpu] n_src=128 (grid read from global memory, chunked FFT): 80x80 ss=2 psf=21, batch 2")
    g = synth.Geometry(80, 0.06, 2, 128, 21, 0.85)
    p = synth.make_problem("X", batch=2, seed=5, geom=g)
    _check(p, range(2))


def test_forward_only_matches_forward_of_gradient_call():
    say("[gpu] forward-only call vs gradient call, C2 batch 2")
    from paper_2606_30620_amd import api
    p = synth.make_problem("C2", batch=2)
    plan = api.plan_for_problem(p)
    lens, ps, lat, nsub = api.device_inputs(p)
    a = api.evaluate(plan, lens, ps, lat, nsub, want_grad=False, want_model=True)
    b = api.evaluate(plan, lens, ps, lat, nsub, want_grad=True, want_model=True)
    torch.cuda.synchronize()
    assert torch.equal(a.loss, b.loss) and torch.equal(a.model, b.model)


@pytest.mark.parametrize("case", ["c2", "ragged"])
def test_ongrid_count_matches_oracle(case):
    """The gradient pass's count of sub-rays on the zero-bordered grid (grid
    coordinates in [-1, n) on both axes) against the oracle's positions; a
    sub-ray within 1e-3 cells of that boundary may fall either way."""
    if case == "c2":
        p = synth.make_problem("C2", batch=2)
    else:
        p = synth.make_problem("X", batch=2, seed=7, geom=synth.Geometry(72, 0.06, 3, 16, 9, 1.2))
    say(f"[gpu] on-grid sub-ray count, {case}")
    plan, res = _run(p)
    n = p.geom.n_src
    for b in range(2):
        got = float(plan.debug_fetch(_lib.DBG_ONGRID, b)[0])
        ref = O.loss_grad_problem(p, b, want_grad=False, return_all=True)
        tx, ty = ref["gx"] * n - 0.5, ref["gy"] * n - 0.5
        on = (tx >= -1) & (tx < n) & (ty >= -1) & (ty < n)
        edge = torch.stack([tx + 1, tx - n, ty + 1, ty - n]).abs().amin(dim=0) < 1e-3
        want, slack = int(on.sum()), int(edge.sum())
        say(f"  sample {b}: gpu {got:.0f} oracle {want} (edge {slack})")
        assert abs(got - want) <= slack


@pytest.mark.parametrize("npix, flags", [(10, 0), (10, 1), (52, 0), (52, 1)])
def test_small_mask_parity(npix, flags):
    """Masks of 10 (fewer than K + 1: status bit 4) and 52 pixels, where
    neighbouring nodes share an order statistic and floor(h_k) + 1 exceeds
    floor(h_{k+1}): every output against the oracle, with the histogram
    selection and with the radix selection (flags = 1)."""
    say(f"[gpu] mask of {npix} pixels, {'radix' if flags else 'histogram'} selection: C1 geometry")
    p = synth.make_problem("C1")
    m = np.zeros_like(p.mask)
    m.reshape(-1)[500:500 + npix] = 1
    p.mask = m
    plan, res, _ = _check(p, [0], flags=flags)
    st = int(res.status[0])
    assert bool(st & 4) == (npix < 23), st
    assert math.isfinite(float(res.loss[0]))


def test_autograd_function_scales_gradients():
    say("[gpu] RTULoss autograd: backward = gradients x grad_output")
    from paper_2606_30620_amd import api
    p = synth.make_problem("C2", batch=2)
    plan = api.plan_for_problem(p)
    lens, ps, lat, nsub = api.device_inputs(p)
    lens.requires_grad_(True)
    ps.requires_grad_(True)
    lat.requires_grad_(True)
    loss = api.RTULoss.apply(lens, ps, lat, plan, nsub)
    (loss * torch.tensor([2.0, -0.5], dtype=torch.float64, device=loss.device)).sum().backward()
    r = api.evaluate(plan, lens.detach(), ps.detach(), lat.detach(), nsub)
    torch.cuda.synchronize()
    # two calls differ at rounding level only (float atomics sum in any order)
    def close(a, b):
        return float((a - b).abs().max()) <= 1e-4 * float(b.abs().max())
    assert close(lens.grad[0], 2.0 * r.grad_lens[0]) and close(lens.grad[1], -0.5 * r.grad_lens[1])
    assert close(ps.grad[0], 2.0 * r.grad_ps[0])
    assert close(lat.grad[1], -0.5 * r.grad_latent[1])


def test_replay_is_deterministic():
    say("[gpu] replay: two identical C2 calls (batch 4) give bitwise-equal results")
    from paper_2606_30620_amd import api
    p = synth.make_problem("C2", batch=4)
    plan = api.plan_for_problem(p)
    lens, ps, lat, nsub = api.device_inputs(p)
    a = api.evaluate(plan, lens, ps, lat, nsub, want_model=True)
    b = api.evaluate(plan, lens, ps, lat, nsub, want_model=True)
    torch.cuda.synchronize()
    for name in ("loss", "model", "grad_lens", "grad_ps", "grad_latent"):
        assert torch.equal(getattr(a, name), getattr(b, name)), name


@pytest.mark.parametrize("case", ["c2", "subhalo", "ragged", "wide"])
def test_radix_selection_matches_histogram_selection(case):
    """The bounded-pass radix select (the fallback for clustered or tied
    masked rays) picks exactly the rays of the histogram + counting select:
    forcing it for every sample leaves every output bit-identical, and the
    forced run agrees with the oracle.  "wide": C3 seed 325, 29859 masked
    rays, above the size from which the prep workgroups are 1024 wide."""
    from paper_2606_30620_amd import _lib
    if case == "c2":
        p = synth.make_problem("C2", batch=2)
    elif case == "wide":
        p = synth.make_problem("C3", batch=2, seed=325)
        assert int(p.mask.sum()) >= 12000
    elif case == "subhalo":
        p = synth.make_problem("X", batch=2, seed=11,
                               geom=synth.Geometry(96, 0.05, 2, 64, 15, 1.0, n_sub_max=3, tnfw_tau=10.0))
    else:
        p = synth.make_problem("X", batch=2, seed=7, geom=synth.Geometry(72, 0.06, 3, 16, 9, 1.2))
    say(f"[gpu] radix vs histogram selection: {case}")
    plan0, r0 = _run(p)
    plan1, r1 = _run(p, flags=_lib.GEOM_RADIX_SELECT)
    for name in ("loss", "chi2_mask", "status", "grad_lens", "grad_ps", "grad_latent", "model"):
        a, b = getattr(r0, name), getattr(r1, name)
        assert torch.equal(a, b), name
    for b in range(p.batch):
        s0 = plan0.debug_fetch(_lib.DBG_SELECT, b)
        s1 = plan1.debug_fetch(_lib.DBG_SELECT, b)
        assert np.array_equal(s0, s1)
    _check(p, [0], flags=_lib.GEOM_RADIX_SELECT)


@pytest.mark.parametrize("seed", [303, 319, 325])
def test_c3_full_size_parity(seed):
    """C3 at full size: 400x400 with 3x3 sub-rays (1.44M rays per sample),
    128x128 source, 31x31 PSF and truncated-NFW subhaloes (seed 303: 9,
    319: 10 = the maximum, 325: 1); batch 4 in one launch, first and last
    samples compared element by element with the oracle."""
    p = synth.make_problem("C3", batch=4, seed=seed)
    say(f"[gpu] C3 400x400 ss=3 n_src=128 psf=31, seed {seed}, {int(p.n_sub[0])} truncated NFW, batch 4")
    _check(p, [0, 3])


def test_c4_full_size_parity():
    """C4 at full size in its launch configuration: 512x512 with 4x4 sub-rays
    (4.2M rays per sample), 256x256 source (chunked FFT, global source grid),
    64 samples in one launch; samples 0 and 63 compared with the oracle."""
    say("[gpu] C4 512x512 ss=4 n_src=256 psf=21, batch 64, samples 0 and 63")
    p = synth.make_problem("C4", batch=64)
    _check(p, [0, 63])
