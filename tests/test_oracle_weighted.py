"""Pins of the oracle's weighted RTU grid (Sec. 6.3: rays weighted when the
eCDFs are built): unit weights give the type-7 quantiles, integer weights give
the quantiles of the rays replicated that many times, zero weights drop rays,
a hand example, and FP64 central differences of the weighted loss."""
import numpy as np
import pytest
import torch

from oracle import rtu_oracle as O
from paper_2606_30620_amd import synth

T = lambda a: torch.as_tensor(np.asarray(a), dtype=torch.float64)


def test_hand_example():
    # sorted: 1 (weight 2), 2 (weight 1), 3 (weight 1) -> the replicated list 1, 1, 2, 3
    z, w = T([3.0, 1.0, 2.0]), T([1.0, 2.0, 1.0])
    u = T([0.0, 0.25, 0.5, 0.9, 1.0])
    q, i0, i1 = O.quantiles_weighted(z, w, u)
    # h = 3u: 0 -> 1; 0.75 -> 1; 1.5 -> (1 + 2)/2; 2.7 -> 2 + 0.7; 3 -> 3
    assert torch.allclose(q, T([1.0, 1.0, 1.5, 2.7, 3.0]), atol=1e-15)
    assert i0.tolist() == [1, 1, 1, 2, 0] and i1.tolist() == [1, 1, 2, 0, 0]


@pytest.mark.parametrize("seed", [0, 1])
def test_unit_weights_are_type7(seed):
    rng = np.random.default_rng(seed)
    z = T(np.round(rng.standard_normal(301), 1))        # many ties
    u = O.chebyshev_nodes()
    a = O.quantiles_type7(z, u)
    b = O.quantiles_weighted(z, torch.ones_like(z), u)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])


@pytest.mark.parametrize("seed", [2, 3])
def test_integer_weights_replicate_rays(seed):
    rng = np.random.default_rng(seed)
    z = T(np.round(rng.standard_normal(120), 2))
    k = rng.integers(0, 5, 120)
    k[0] = 3
    u = O.chebyshev_nodes()
    q, i0, i1 = O.quantiles_weighted(z, T(k.astype(float)), u)
    rep = torch.repeat_interleave(torch.arange(120), torch.as_tensor(k))
    qr, j0, j1 = O.quantiles_type7(z[rep], u)
    assert torch.allclose(q, qr, atol=1e-15)
    # the replicated copies of a ray are adjacent in the stable sort, so the
    # picked copy is a copy of the picked ray
    assert torch.equal(rep[j0], i0) and torch.equal(rep[j1], i1)
    assert bool((k[i0.numpy()] > 0).all() and (k[i1.numpy()] > 0).all())    # weight 0: never picked


def test_weighted_transform_equals_transform_of_replicated_rays():
    rng = np.random.default_rng(4)
    bxm, bym = T(rng.standard_normal(200) * 0.7), T(rng.gamma(2.0, 0.4, 200))
    k = rng.integers(1, 4, 200)
    a = O.build_transform(bxm, bym, weights=T(k.astype(float)))
    rep = torch.repeat_interleave(torch.arange(200), torch.as_tensor(k))
    b = O.build_transform(bxm[rep], bym[rep])
    for key in ("mu",):
        assert all(abs(float(x - y)) < 1e-13 for x, y in zip(a[key], b[key]))
    assert abs(float(a["s"] - b["s"])) < 1e-13
    for ax in range(2):
        assert torch.allclose(a["X"][ax], b["X"][ax], atol=1e-12)
        assert torch.allclose(a["S"][ax], b["S"][ax], rtol=1e-10)
    zs = T(np.linspace(-3, 3, 101))
    ga, gb = O.rtu_transform(zs, zs, a), O.rtu_transform(zs, zs, b)
    assert torch.allclose(ga[0], gb[0], atol=1e-12) and torch.allclose(ga[1], gb[1], atol=1e-12)


def _weighted_c1():
    p = synth.make_problem("C1")
    obs = O.obs_from_problem(p)
    img = np.abs(p.image.astype(np.float64))
    obs["ray_weights"] = T(img / img[p.mask.astype(bool)].mean())     # brightness, mean 1 over the mask
    return p, obs


def test_weighted_loss_differs_and_unit_weights_do_not():
    p, obs = _weighted_c1()
    lens, ps, w = (p.lens[0].astype(np.float64), p.ps[0].astype(np.float64), p.latent[0].astype(np.float64))
    a = O.loss_grad(lens, ps, w, O.obs_from_problem(p), want_grad=False)
    b = O.loss_grad(lens, ps, w, obs, want_grad=False)
    c = O.loss_grad(lens, ps, w, dict(obs, ray_weights=torch.ones(p.geom.n_img, p.geom.n_img, dtype=torch.float64)),
                    want_grad=False)
    assert float(c["loss"]) == float(a["loss"])
    assert abs(float(b["loss"]) - float(a["loss"])) > 1e-6 * abs(float(a["loss"]))


def test_weighted_gradient_matches_central_differences():
    p, obs = _weighted_c1()
    lens, ps, w = (p.lens[0].astype(np.float64), p.ps[0].astype(np.float64), p.latent[0].astype(np.float64))
    r = O.loss_grad(lens, ps, w, obs)
    L = lambda l_: float(O.loss_grad(l_, ps, w, obs, want_grad=False)["loss"])
    for i in range(lens.size):
        ok = False
        for h in (1e-6, 2.5e-7, 6e-8):
            lp, lm = lens.copy(), lens.copy()
            lp[i] += h
            lm[i] -= h
            f0, fp, fm = L(lens), L(lp), L(lm)
            fwd, bwd, cen = (fp - f0) / h, (f0 - fm) / h, (fp - fm) / (2 * h)
            scale = max(abs(cen), 1e-3 * float(r["grad_lens"].abs().max()))
            if abs(fwd - bwd) < 1e-3 * scale:
                assert abs(cen - float(r["grad_lens"][i])) < 2e-4 * scale, (i, cen, float(r["grad_lens"][i]))
                ok = True
                break
        assert ok, f"lens parameter {i}: no kink-free step found"
