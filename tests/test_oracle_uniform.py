"""Pins of the oracle's uniform-grid mode (Sec. 2.1: the source grid spans the
smallest square box that holds the masked rays) against brute force, the RTU
grid where the two coincide (Sec. 6.1), and FP64 central differences."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import rtu_oracle as O
from paper_2606_30620_amd import synth
from tests.test_oracle_pipeline import _zero_mass_obs

T = lambda a: torch.as_tensor(np.asarray(a), dtype=torch.float64)


def _box_brute(xs, ys):
    """The reading written out with Python loops: extremes by scanning (lowest
    index wins a tie for the minimum, highest index for the maximum), side =
    the larger range (x on a tie), centred on both ranges."""
    def ext(z):
        imin = imax = 0
        for i, v in enumerate(z):
            if v < z[imin]:
                imin = i
            if v >= z[imax]:
                imax = i
        return imin, imax
    (ax0, ax1), (ay0, ay1) = ext(xs), ext(ys)
    rx, ry = xs[ax1] - xs[ax0], ys[ay1] - ys[ay0]
    side = rx if rx >= ry else ry
    lo = (0.5 * (xs[ax0] + xs[ax1]) - 0.5 * side, 0.5 * (ys[ay0] + ys[ay1]) - 0.5 * side)
    return lo, side, ((ax0, ax1), (ay0, ay1))


@pytest.mark.parametrize("seed, sx, sy", [(1, 1.0, 0.4), (2, 0.3, 1.2), (3, 1.0, 1.0)])
def test_box_matches_brute_force(seed, sx, sy):
    rng = np.random.default_rng(seed)
    xs = list(np.round(rng.standard_normal(57) * sx, 2))    # rounded: ties among the extremes
    ys = list(np.round(rng.standard_normal(57) * sy, 2))
    xs[10] = xs[40] = max(xs) + 0.5                         # a tied maximum
    ys[3] = ys[50] = min(ys) - 0.25                         # a tied minimum
    box = O.uniform_box_of(T(xs), T(ys))
    lo, side, idx = _box_brute(xs, ys)
    assert abs(float(box["side"]) - side) < 1e-15
    assert abs(float(box["lo"][0]) - lo[0]) < 1e-15 and abs(float(box["lo"][1]) - lo[1]) < 1e-15
    for ax in range(2):
        assert int(box["idx"][ax][0]) == idx[ax][0] and int(box["idx"][ax][1]) == idx[ax][1]
    assert box["status"] == 0
    # every ray inside, the longer axis spanned exactly
    g = [(T(v) - box["lo"][a]) / box["side"] for a, v in enumerate((xs, ys))]
    assert all(bool((x >= -1e-15).all() and (x <= 1 + 1e-15).all()) for x in g)
    assert any(abs(float(x.min())) < 1e-15 and abs(float(x.max()) - 1) < 1e-15 for x in g)


def test_box_derivative_is_a_selection():
    """d side / d ray and d lo / d ray fall on the extreme rays only, with the
    weights of the reading (x range the longer: side = x_max - x_min,
    lo_y = (y_min + y_max)/2 - side/2)."""
    rng = np.random.default_rng(7)
    xs = T(rng.uniform(-2.0, 2.0, 40)).requires_grad_(True)
    ys = T(rng.uniform(-0.5, 0.5, 40)).requires_grad_(True)
    box = O.uniform_box_of(xs, ys)
    (ix0, ix1), (iy0, iy1) = [(int(a), int(b)) for a, b in box["idx"]]
    gx, gy = torch.autograd.grad(box["side"], (xs, ys), retain_graph=True)
    want = torch.zeros(40, dtype=torch.float64)
    want[ix1], want[ix0] = 1.0, -1.0
    assert torch.equal(gx, want) and not bool(gy.any())
    gx, gy = torch.autograd.grad(box["lo"][1], (xs, ys))
    wx = torch.zeros(40, dtype=torch.float64)
    wx[ix1], wx[ix0] = -0.5, 0.5
    wy = torch.zeros(40, dtype=torch.float64)
    wy[iy0] += 0.5
    wy[iy1] += 0.5
    assert torch.equal(gx, wx) and torch.equal(gy, wy)


def test_uniform_mode_equals_rtu_grid_on_uniform_rays():
    """Zero mass and a diagonal mask: the masked rays are equispaced with equal
    ranges, so the square box is the rays' bounding box, which is also what
    the RTU transform maps onto [0, 1] (Sec. 6.1)."""
    obs = _zero_mass_obs()
    n, pix = obs["n_img"], obs["pix"]
    lens = T([0.0, 0.1, 0.05, 0.0, 0.0, 0.0, 0.0])
    rng = np.random.default_rng(4)
    w = T(rng.standard_normal((16, 16)))
    ps = T(synth.matern_ps_for_k0(4.0, 1.0))
    a = O.forward(lens, ps, w, obs, return_all=True)
    b = O.forward(lens, ps, w, dict(obs, grid="uniform"), return_all=True)
    lo = -0.5 * (n - 1) * pix
    assert abs(float(b["transform"]["side"]) - (n - 1) * pix) < 1e-14
    assert abs(float(b["transform"]["lo"][0]) - lo) < 1e-14 and abs(float(b["transform"]["lo"][1]) - lo) < 1e-14
    assert torch.allclose(a["gx"], b["gx"], atol=1e-12) and torch.allclose(a["gy"], b["gy"], atol=1e-12)
    assert torch.allclose(a["model"], b["model"], atol=1e-12)


def test_uniform_mode_on_a_rectangular_mask_pads_the_short_axis():
    """A mask twice as wide as tall: the box is square with the x range as its
    side, and the masked rays fill the middle half of it along y."""
    obs = _zero_mass_obs(diag=False)        # mask rows 10..29, columns 5..39
    lens = T([0.0, 0.1, 0.05, 0.0, 0.0, 0.0, 0.0])
    rng = np.random.default_rng(5)
    out = O.forward(lens, T(synth.matern_ps_for_k0(4.0, 1.0)), T(rng.standard_normal((16, 16))),
                    dict(obs, grid="uniform"), return_all=True)
    m = obs["mask"].reshape(-1).bool()
    gx, gy = out["gx"][m, 0], out["gy"][m, 0]
    assert abs(float(gx.min())) < 1e-14 and abs(float(gx.max()) - 1.0) < 1e-14
    span = 19.0 / 34.0
    assert abs(float(gy.min()) - (0.5 - span / 2)) < 1e-13 and abs(float(gy.max()) - (0.5 + span / 2)) < 1e-13


def test_degenerate_mask_sets_status_bit_4():
    obs = _zero_mass_obs()
    mask = torch.zeros_like(obs["mask"])
    mask[3, 7] = 1
    lens = T([0.8, 0.1, 0.05, 0.0, 0.0, 0.0, 0.0])
    out = O.forward(lens, T(synth.matern_ps_for_k0(4.0, 1.0)), T(np.zeros((16, 16))),
                    dict(obs, grid="uniform", mask=mask))
    assert out["status"] & O.ST_MASK_SMALL and bool(torch.isfinite(out["loss"]))


def test_uniform_mode_gradient_matches_central_differences():
    """The exact derivative of the uniform-grid loss, box included, against
    FP64 central differences (the extremes change identity only at kinks, so a
    step whose one-sided differences disagree is retried smaller)."""
    p = synth.make_problem("C1")
    p = dataclasses.replace(p, geom=dataclasses.replace(p.geom, uniform=True))
    obs = O.obs_from_problem(p)
    assert obs["grid"] == "uniform"
    lens, ps, w = (p.lens[0].astype(np.float64), p.ps[0].astype(np.float64), p.latent[0].astype(np.float64))
    r = O.loss_grad(lens, ps, w, obs)
    L = lambda l_, p_, w_: float(O.loss_grad(l_, p_, w_, obs, want_grad=False)["loss"])
    for i in range(lens.size):
        ok = False
        for h in (1e-6, 2.5e-7, 6e-8):
            lp, lm = lens.copy(), lens.copy()
            lp[i] += h
            lm[i] -= h
            f0, fp, fm = L(lens, ps, w), L(lp, ps, w), L(lm, ps, w)
            fwd, bwd, cen = (fp - f0) / h, (f0 - fm) / h, (fp - fm) / (2 * h)
            scale = max(abs(cen), 1e-3 * float(r["grad_lens"].abs().max()))
            if abs(fwd - bwd) < 1e-3 * scale:
                assert abs(cen - float(r["grad_lens"][i])) < 2e-4 * scale, (i, cen, float(r["grad_lens"][i]))
                ok = True
                break
        assert ok, f"lens parameter {i}: no kink-free step found"
    for i in range(4):
        hp = 1e-6 * max(1.0, abs(ps[i]))
        pp, pm = ps.copy(), ps.copy()
        pp[i] += hp
        pm[i] -= hp
        cen = (L(lens, pp, w) - L(lens, pm, w)) / (2 * hp)
        assert abs(cen - float(r["grad_ps"][i])) < 1e-5 * max(abs(cen), 1.0)
