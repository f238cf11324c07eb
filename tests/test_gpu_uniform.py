"""Parity of the HIP path in uniform-grid mode (RTU_GEOM_UNIFORM: the source
grid on the smallest square box of the masked rays, Sec. 2.1) with the FP64
oracle's uniform mode: loss, images and gradients to the tolerances of the
RTU parity tests, the box and the rays standing for its extremes."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import rtu_oracle as O
from paper_2606_30620_amd import _lib, synth
from tests.gpu_helpers import TIE_REL, compare, say

pytestmark = pytest.mark.gpu


def _uniform(p):
    return dataclasses.replace(p, geom=dataclasses.replace(p.geom, uniform=True))


def _check(p, samples):
    from paper_2606_30620_amd import api
    plan = api.plan_for_problem(p)
    lens, ps, lat, nsub = api.device_inputs(p)
    res = api.evaluate(plan, lens, ps, lat, nsub, want_grad=True, want_model=True)
    torch.cuda.synchronize()
    xc, yc = O.pixel_centres(p.geom.n_img, float(np.float32(p.geom.pixel_scale)))
    m = torch.as_tensor(p.mask.reshape(-1).astype(bool))
    for b in samples:
        ref = O.loss_grad_problem(p, b, want_grad=True, return_all=True)
        box = ref["transform"]
        sel = plan.debug_fetch(_lib.DBG_SELECT, b)
        std = plan.debug_fetch(_lib.DBG_STD, b)
        assert int(res.status[b]) == ref["status"], (int(res.status[b]), ref["status"])
        side = float(box["side"].detach())
        d_box = max(abs(std[0] - float(box["lo"][0].detach())), abs(std[1] - float(box["lo"][1].detach())),
                    abs(std[2] - side)) / side
        assert d_box < 1e-5, ("box", std, box["lo"], side)
        lens_b = torch.as_tensor(p.lens[b].astype(np.float64))
        bxm, bym = O.ray_shoot(xc[m], yc[m], lens_b, int(p.n_sub[b]), p.geom.tnfw_tau)
        picks, same = [], True
        for ax, z in enumerate((bxm.numpy(), bym.numpy())):
            got = (int(sel[ax][0]), int(sel[ax][1]))
            want = (int(box["idx"][ax][0]), int(box["idx"][ax][1]))
            for g_, w_ in zip(got, want):
                if g_ != w_:
                    same = False
                    assert abs(z[g_] - z[w_]) <= TIE_REL * float(z.max() - z.min()), (ax, g_, w_)
            picks.append(got)
        if not same:
            ref = O.loss_grad_problem(p, b, want_grad=True, return_all=True, picks=picks)
        out = compare(plan, p, b, res, ref, check_stages=False)
        say(f"  sample {b}: box {d_box:.1e} " + ", ".join(f"{k}={v:.2e}" if isinstance(v, float) else f"{k}={v}"
                                                       for k, v in out.items()))


def test_uniform_c1():
    say("[gpu] uniform grid: C1 64x64 ss=1 n_src=32")
    _check(_uniform(synth.make_problem("C1")), [0])


def test_uniform_c2_batch():
    say("[gpu] uniform grid: C2 200x200 ss=4 n_src=64, batch 3")
    _check(_uniform(synth.make_problem("C2", batch=3)), range(3))


def test_uniform_ragged_subhaloes_and_global_grid():
    say("[gpu] uniform grid: 72x72 ss=3 n_src=16 psf=9 batch 2; 80x80 ss=2 n_src=128 with 2 subhaloes")
    g = synth.Geometry(72, 0.06, 3, 16, 9, 1.2, uniform=True)
    _check(synth.make_problem("X", batch=2, seed=7, geom=g), range(2))
    g = synth.Geometry(80, 0.06, 2, 128, 21, 0.85, n_sub_max=2, tnfw_tau=10.0, uniform=True)
    _check(synth.make_problem("X", batch=2, seed=9, geom=g), range(2))


def test_uniform_flag_selects_the_uniform_model():
    """On a problem whose RTU and uniform-grid losses differ, each GPU mode
    gives the oracle's loss of the same mode (a flag that did nothing would
    fail here)."""
    from paper_2606_30620_amd import api
    p = synth.make_problem("C1")
    pu = _uniform(p)
    outs = []
    for q in (p, pu):
        plan = api.plan_for_problem(q)
        lens, ps, lat, nsub = api.device_inputs(q)
        outs.append(float(api.evaluate(plan, lens, ps, lat, nsub, want_grad=False).loss[0]))
    ref_rtu = float(O.loss_grad_problem(p, 0, want_grad=False)["loss"])
    ref_uni = float(O.loss_grad_problem(pu, 0, want_grad=False)["loss"])
    assert abs(ref_rtu - ref_uni) > 1e-3 * abs(ref_rtu)
    assert abs(outs[0] - ref_rtu) <= 1e-4 * abs(ref_rtu) and abs(outs[1] - ref_uni) <= 1e-4 * abs(ref_uni)


def test_uniform_one_pixel_mask_sets_status_bit_4():
    from paper_2606_30620_amd import api
    p = _uniform(synth.make_problem("C1"))
    mask = np.zeros_like(p.mask)
    mask[20, 30] = 1
    p = dataclasses.replace(p, mask=mask)
    plan = api.plan_for_problem(p)
    lens, ps, lat, nsub = api.device_inputs(p)
    res = api.evaluate(plan, lens, ps, lat, nsub, want_grad=True)
    torch.cuda.synchronize()
    ref = O.loss_grad_problem(p, 0, want_grad=False)
    assert int(res.status[0]) & O.ST_MASK_SMALL and ref["status"] & O.ST_MASK_SMALL
    assert abs(float(res.loss[0]) - float(ref["loss"])) <= 1e-4 * abs(float(ref["loss"]))
    assert bool(torch.isfinite(res.grad_lens).all())
