"""Pins of the oracle's lens light (App. A, Multi Gaussian Expansion) against
mathematics that does not share its formula: scipy's bivariate normal density,
the flux integral, the orientation shared with the mass model, and the
image model's response to the light."""
import math

import numpy as np
import pytest
import torch
from scipy import stats

from oracle import rtu_oracle as O
from paper_2606_30620_amd import synth

T = lambda a: torch.tensor(a, dtype=torch.float64)


def _components(rng, n):
    out = []
    for _ in range(n):
        q, phi = rng.uniform(0.4, 0.95), rng.uniform(0.0, math.pi)
        e = (1 - q) / (1 + q)
        out += [rng.uniform(0.3, 2.0), rng.uniform(0.1, 1.0), e * math.cos(2 * phi), e * math.sin(2 * phi),
                rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2)]
    return np.array(out)


def test_mge_light_is_a_sum_of_bivariate_normal_densities():
    """Component n is A_n sigma_n^2 times the density of a bivariate normal with
    mean (x_n, y_n), standard deviations sigma_n/sqrt(q_n) along the position
    angle and sigma_n sqrt(q_n) across it."""
    rng = np.random.default_rng(7)
    light = _components(rng, 3)
    x, y = rng.uniform(-1.5, 1.5, 200), rng.uniform(-1.5, 1.5, 200)
    want = np.zeros_like(x)
    for n in range(3):
        A, sig, e1, e2, xc, yc = light[6 * n:6 * n + 6]
        e = math.hypot(e1, e2)
        q, phi = (1 - e) / (1 + e), 0.5 * math.atan2(e2, e1)
        u = np.array([math.cos(phi), math.sin(phi)])
        v = np.array([-math.sin(phi), math.cos(phi)])
        cov = sig * sig * (np.outer(u, u) / q + np.outer(v, v) * q)
        want += A * sig * sig * stats.multivariate_normal(mean=[xc, yc], cov=cov).pdf(np.stack([x, y], 1))
    got = O.mge_light(T(x), T(y), T(light)).numpy()
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("q", [1.0, 0.6])
def test_mge_light_flux(q):
    """The integral of A/(2 pi) exp(-rho^2/(2 sigma^2)) over the plane is A sigma^2
    for every axis ratio (rho^2 = q x'^2 + y'^2/q keeps areas)."""
    A, sig, phi = 1.7, 0.3, 0.4
    e = (1 - q) / (1 + q)
    light = T([A, sig, e * math.cos(2 * phi), e * math.sin(2 * phi), 0.05, -0.02])
    h = 0.004
    c = torch.arange(-3.0, 3.0 + h / 2, h, dtype=torch.float64)
    yy, xx = torch.meshgrid(c, c, indexing="ij")
    flux = float(O.mge_light(xx.reshape(-1), yy.reshape(-1), light).sum()) * h * h
    assert abs(flux - A * sig * sig) < 1e-9 * A * sig * sig


def test_mge_light_orientation_follows_the_mass_convention():
    """At position angle 0 the light falls off more slowly along x (q multiplies
    x'^2, as in the SIE's elliptical radius); at pi/2 along y."""
    q = 0.5
    e = (1 - q) / (1 + q)
    d = T([0.3])
    z = T([0.0])
    for phi, along_x in ((0.0, True), (0.5 * math.pi, False)):
        light = T([1.0, 0.4, e * math.cos(2 * phi), e * math.sin(2 * phi), 0.0, 0.0])
        lx, ly = float(O.mge_light(d, z, light)), float(O.mge_light(z, d, light))
        assert (lx > ly) == along_x


def test_light_adds_to_every_sub_ray_before_the_psf():
    """With a zero source (tiny GP amplitude) the model image is the PSF applied
    to the sub-ray mean of the light."""
    g = synth.Geometry(24, 0.1, 2, 16, 5, 1.0, n_gauss=2)
    p = synth.make_problem("C2", batch=1, geom=g)
    obs = O.obs_from_problem(p)
    lens = p.lens[0].astype(np.float64)
    ps = p.ps[0].astype(np.float64).copy()
    ps[0] = 1e-30
    w = np.zeros((16, 16))
    out = O.forward(T(lens), T(ps), T(w), obs, return_all=True)
    xr, yr = O.subray_positions(24, obs["pix"], 2)
    light = O.mge_light(xr, yr, T(lens[-12:])).mean(dim=1).reshape(24, 24)
    # the GP source of a zero latent is the softplus of zero, a constant
    # s0 ln 2 in the grid; subtract its bilinear image
    ref = O.forward(T(lens[:7]), T(ps), T(w), dict(obs, n_gauss=0), return_all=True)
    np.testing.assert_allclose((out["u"] - ref["u"]).numpy(), light.numpy(), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(out["model"].numpy(),
                               O.psf_convolve(out["u"], obs["psf"]).numpy(), rtol=1e-12, atol=1e-15)


def test_light_domain_status():
    g = synth.Geometry(24, 0.1, 1, 16, 5, 1.0, n_gauss=1)
    p = synth.make_problem("C2", batch=1, geom=g)
    obs = O.obs_from_problem(p)
    lens = p.lens[0].astype(np.float64).copy()
    assert not O.loss_grad(lens, p.ps[0], p.latent[0], obs, want_grad=False)["status"] & O.ST_DOMAIN
    lens[-5] = -0.1                      # sigma <= 0
    assert O.loss_grad(lens, p.ps[0], p.latent[0], obs, want_grad=False)["status"] & O.ST_DOMAIN


def test_light_gradient_matches_central_differences():
    """The lens-light part of the exact gradient against FP64 central
    differences (the light is smooth: no kinks)."""
    g = synth.Geometry(32, 0.08, 2, 16, 7, 1.2, n_gauss=2)
    p = synth.make_problem("C2", batch=1, geom=g)
    obs = O.obs_from_problem(p)
    lens = p.lens[0].astype(np.float64)
    ps = p.ps[0].astype(np.float64)
    w = p.latent[0].astype(np.float64)
    r = O.loss_grad(lens, ps, w, obs)
    L = lambda l_: float(O.loss_grad(l_, ps, w, obs, want_grad=False)["loss"])
    for i in range(7, lens.size):
        h = 1e-6
        lp, lm = lens.copy(), lens.copy()
        lp[i] += h
        lm[i] -= h
        cen = (L(lp) - L(lm)) / (2 * h)
        g_ = float(r["grad_lens"][i])
        assert abs(cen - g_) < 1e-5 * max(abs(cen), 1.0), (i, cen, g_)
