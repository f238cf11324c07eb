"""Pins of the oracle's elliptical power law (App. A.1, eq. A1) against the
deflection integrals of its convergence (Keeton 2001: one-dimensional
integrals of kappa over homoeoids, evaluated by adaptive quadrature with the
integrable end-point singularity as a weight), the SIE at slope 2, the
circular power law, scipy's hypergeometric function, divergence = 2 kappa,
zero curl, homogeneity, and FP64 central differences of the loss."""
import math

import numpy as np
import pytest
import torch
from scipy import integrate, special

from oracle import rtu_oracle as O
from paper_2606_30620_amd import synth

T = lambda a: torch.as_tensor(np.asarray(a), dtype=torch.float64)


def kappa(x, y, te, e1, e2, x0, y0, g):
    """Eq. (A1) written out: rho^2 = q x'^2 + y'^2/q in the frame of angle phi."""
    e = math.hypot(e1, e2)
    q, phi = (1 - e) / (1 + e), 0.5 * math.atan2(e2, e1)
    xp = math.cos(phi) * (x - x0) + math.sin(phi) * (y - y0)
    yp = -math.sin(phi) * (x - x0) + math.cos(phi) * (y - y0)
    rho = math.sqrt(q * xp * xp + yp * yp / q)
    return 0.5 * (3 - g) * (te / rho) ** (g - 1)


def alpha_keeton(x, y, te, e1, e2, x0, y0, g):
    """alpha'_x = q x' J_0, alpha'_y = q y' J_1 with
    J_n = int_0^1 kappa(xi(u)^2) [1 - (1 - q^2) u]^-(n + 1/2) du,
    xi(u)^2 = u (x'^2 + y'^2 / (1 - (1 - q^2) u)), in the lens frame, where
    kappa(xi^2) = (3-g)/2 te^(g-1) (q xi^2)^(-(g-1)/2); rotated back."""
    e = math.hypot(e1, e2)
    q, phi = (1 - e) / (1 + e), 0.5 * math.atan2(e2, e1)
    c, s = math.cos(phi), math.sin(phi)
    xp, yp = c * (x - x0) + s * (y - y0), -s * (x - x0) + c * (y - y0)
    a = -(g - 1) / 2
    pref = 0.5 * (3 - g) * te ** (g - 1) * q ** a

    def J(nn):
        f = lambda u: (xp * xp + yp * yp / (1 - (1 - q * q) * u)) ** a / (1 - (1 - q * q) * u) ** (nn + 0.5)
        return pref * integrate.quad(f, 0.0, 1.0, weight="alg", wvar=(a, 0.0), epsabs=1e-14, epsrel=1e-13)[0]

    axp, ayp = q * xp * J(0), q * yp * J(1)
    return c * axp - s * ayp, s * axp + c * ayp


def _epl(x, y, *p):
    return O.epl_deflection(T(x), T(y), *[T(v) for v in p])


PTS = [(0.9, 0.3), (-0.4, 1.1), (0.05, -0.7), (-1.3, -0.6), (0.2, 0.01)]


@pytest.mark.parametrize("g", [1.5, 1.85, 2.0, 2.25, 2.7])
@pytest.mark.parametrize("e1, e2", [(0.0, 0.0), (0.25, 0.0), (0.18, -0.3), (-0.05, 0.45)])
def test_matches_keeton_integrals(g, e1, e2):
    te, x0, y0 = 1.2, 0.07, -0.04
    for x, y in PTS:
        ax, ay = _epl([x], [y], te, e1, e2, x0, y0, g)
        kx, ky = alpha_keeton(x, y, te, e1, e2, x0, y0, g)
        assert abs(float(ax[0]) - kx) < 1e-10 and abs(float(ay[0]) - ky) < 1e-10, (g, e1, e2, x, y)


@pytest.mark.parametrize("e1, e2", [(0.0, 0.0), (0.3, 0.1), (0.0004, -0.0002), (-0.5, 0.2)])
def test_slope_two_is_the_sie(e1, e2):
    rng = np.random.default_rng(1)
    x, y = rng.uniform(-2, 2, 200), rng.uniform(-2, 2, 200)
    a = _epl(x, y, 1.1, e1, e2, 0.05, 0.02, 2.0)
    b = O.sie_deflection(T(x), T(y), T(1.1), T(e1), T(e2), T(0.05), T(0.02))
    assert torch.allclose(a[0], b[0], atol=1e-12) and torch.allclose(a[1], b[1], atol=1e-12)


@pytest.mark.parametrize("g", [1.4, 2.3])
def test_round_lens_is_the_circular_power_law(g):
    rng = np.random.default_rng(2)
    x, y = rng.uniform(-2, 2, 50), rng.uniform(-2, 2, 50)
    ax, ay = _epl(x, y, 0.9, 0.0, 0.0, 0.0, 0.0, g)
    r = np.hypot(x, y)
    mag = 0.9 ** (g - 1) * r ** (2 - g)       # alpha(r) = M(<r)/(pi r)
    assert np.allclose(ax.numpy(), mag * x / r, atol=1e-13) and np.allclose(ay.numpy(), mag * y / r, atol=1e-13)


def test_series_matches_scipy_hypergeometric():
    """F(w) = 2F1(1, t/2; 2 - t/2; w) on real w (u = 1 or i: the lens axes)."""
    for g in (1.3, 2.0, 2.6):
        t = g - 1
        for e in (0.1, 0.4, 0.7):
            for x, y, sgn in ((1.0, 0.0, -1.0), (0.0, 1.0, 1.0)):
                # on the axes u^2 = +-1, so w = -e u^2 = -+e
                ax, ay = _epl([x], [y], 1.0, e, 0.0, 0.0, 0.0, g)
                lam = math.sqrt(1 - e * e)
                m = abs(x - e * x) if y == 0 else abs(y + e * y)
                F = special.hyp2f1(1.0, t / 2, 2 - t / 2, sgn * e)
                want = lam ** t * m ** (1 - t) * F
                got = float(ax[0]) if y == 0 else float(ay[0])
                assert abs(got - want) < 1e-12 * max(1.0, abs(want)), (g, e, x, y)


@pytest.mark.parametrize("g", [1.7, 2.4])
def test_divergence_is_twice_kappa_and_curl_free(g):
    p = (1.05, 0.2, -0.15, 0.03, 0.01, g)
    h = 1e-5
    for x, y in PTS[:4]:
        axp = _epl([x + h], [y], *p)
        axm = _epl([x - h], [y], *p)
        ayp = _epl([x], [y + h], *p)
        aym = _epl([x], [y - h], *p)
        div = (float(axp[0][0] - axm[0][0]) + float(ayp[1][0] - aym[1][0])) / (2 * h)
        curl = (float(axp[1][0] - axm[1][0]) - float(ayp[0][0] - aym[0][0])) / (2 * h)
        k = kappa(x, y, *p)
        assert abs(div - 2 * k) < 1e-7 * max(1.0, k) and abs(curl) < 1e-7


def test_homogeneity():
    """alpha(x0 + lam d) = lam^(2 - gamma) alpha(x0 + d)."""
    g = 2.35
    p = (1.0, -0.1, 0.3, 0.2, -0.1, g)
    for d in ((0.4, 0.3), (-0.2, 0.9)):
        a1 = _epl([0.2 + d[0]], [-0.1 + d[1]], *p)
        a2 = _epl([0.2 + 2.5 * d[0]], [-0.1 + 2.5 * d[1]], *p)
        f = 2.5 ** (2 - g)
        assert abs(float(a2[0][0]) - f * float(a1[0][0])) < 1e-12 and abs(float(a2[1][0]) - f * float(a1[1][0])) < 1e-12


def test_epl_loss_gradient_matches_central_differences():
    """The exact derivative of the loss with the EPL deflector (slope
    included) against FP64 central differences."""
    p = synth.make_problem("C1")
    obs = dict(O.obs_from_problem(p), lens_model="epl")
    lens = np.concatenate([p.lens[0].astype(np.float64), [2.15]])
    ps, w = p.ps[0].astype(np.float64), p.latent[0].astype(np.float64)
    r = O.loss_grad(lens, ps, w, obs)
    L = lambda l_: float(O.loss_grad(l_, ps, w, obs, want_grad=False)["loss"])
    for i in range(lens.size):
        ok = False
        # (the order statistics make the loss piecewise smooth; a step whose
        # one-sided differences disagree by more than 2e-4 straddles a kink)
        for h in (1e-6, 2.5e-7, 6e-8, 1.5e-8):
            lp, lm = lens.copy(), lens.copy()
            lp[i] += h
            lm[i] -= h
            f0, fp, fm = L(lens), L(lp), L(lm)
            fwd, bwd, cen = (fp - f0) / h, (f0 - fm) / h, (fp - fm) / (2 * h)
            scale = max(abs(cen), 1e-3 * float(r["grad_lens"].abs().max()))
            if abs(fwd - bwd) < 2e-4 * scale:
                assert abs(cen - float(r["grad_lens"][i])) < 2e-4 * scale, (i, cen, float(r["grad_lens"][i]))
                ok = True
                break
        assert ok, f"lens parameter {i}: no kink-free step found"
