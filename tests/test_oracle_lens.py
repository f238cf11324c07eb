"""Pins of the oracle's lens-mass step against mathematics that does not share
its formulas: numerical integration of the convergence (App. A, eqs. A1-A3),
the Poisson equation div alpha = 2 kappa, curl-free fields, high-precision
evaluation and the known limits."""
import math

import mpmath
import numpy as np
import pytest
import torch
from scipy import integrate

from oracle import rtu_oracle as O

T = lambda a: torch.tensor(a, dtype=torch.float64)


def kappa_sie(x, y, the, q, phi, x0=0.0, y0=0.0):
    """Eq. (A1) at gamma = 2: (theta_E/2)/rho, rho^2 = q x'^2 + y'^2/q."""
    c, s = math.cos(phi), math.sin(phi)
    dx, dy = x - x0, y - y0
    xp, yp = c * dx + s * dy, -s * dx + c * dy
    return 0.5 * the / math.sqrt(q * xp * xp + yp * yp / q)


def schramm_alpha(x, y, the, q):
    """Deflection of an elliptical convergence by the one-dimensional integrals of
    Schramm (1990) as written by Keeton (2001): with xi^2 = x^2 + y^2/q^2 and
    kappa(xi), alpha_x = q x J0, alpha_y = q y J1,
    J_n = int_0^1 kappa(xi(u)) / (1 - (1-q^2) u)^(n + 1/2) du,
    xi(u)^2 = u (x^2 + y^2 / (1 - (1-q^2) u)).  Here kappa(xi) = theta_E/(2 sqrt(q) xi).
    u = v^2 removes the integrable 1/sqrt(u) end point."""
    def kap(xi):
        return the / (2.0 * math.sqrt(q) * xi)

    def J(n):
        def f(v):
            u = v * v
            d = 1.0 - (1.0 - q * q) * u
            xi = math.sqrt(u * (x * x + y * y / d))
            return 2.0 * v * kap(xi) / d ** (n + 0.5)
        return integrate.quad(f, 0.0, 1.0, epsabs=1e-14, epsrel=1e-13, limit=200)[0]
    return q * x * J(0), q * y * J(1)


@pytest.mark.parametrize("q", [0.5, 0.8, 0.95])
def test_sie_matches_schramm_integral(q):
    rng = np.random.default_rng(1)
    the = 1.3
    e = (1 - q) / (1 + q)
    for _ in range(6):
        x, y = rng.uniform(-2, 2, 2)
        # axis-aligned lens (phi = 0): e2 = 0, e1 = e
        ax, ay = O.sie_deflection(T(x), T(y), T(the), T(e), T(0.0), T(0.0), T(0.0))
        rx, ry = schramm_alpha(x, y, the, q)
        assert abs(float(ax) - rx) < 1e-10 and abs(float(ay) - ry) < 1e-10, (x, y, q)


def _div_curl(fn, x, y, h=1e-5):
    axp, ayp = fn(T(x + h), T(y))
    axm, aym = fn(T(x - h), T(y))
    bxp, byp = fn(T(x), T(y + h))
    bxm, bym = fn(T(x), T(y - h))
    dxx = (float(axp) - float(axm)) / (2 * h)
    dyx = (float(ayp) - float(aym)) / (2 * h)
    dxy = (float(bxp) - float(bxm)) / (2 * h)
    dyy = (float(byp) - float(bym)) / (2 * h)
    return dxx + dyy, dyx - dxy


def test_sie_poisson_and_curl_free_rotated():
    rng = np.random.default_rng(2)
    the, q, phi, x0, y0 = 1.1, 0.7, 0.6, 0.05, -0.03
    e = (1 - q) / (1 + q)
    e1, e2 = e * math.cos(2 * phi), e * math.sin(2 * phi)
    fn = lambda x, y: O.sie_deflection(x, y, T(the), T(e1), T(e2), T(x0), T(y0))
    for _ in range(8):
        x, y = rng.uniform(-1.8, 1.8, 2)
        div, curl = _div_curl(fn, x, y)
        assert abs(div - 2 * kappa_sie(x, y, the, q, phi, x0, y0)) < 1e-6
        assert abs(curl) < 1e-6


def test_sie_sis_limit_and_einstein_ring_mean_kappa():
    # q -> 1: |alpha| = theta_E everywhere (singular isothermal sphere)
    x, y = T([0.3, -1.2, 0.7]), T([0.4, 0.5, -2.0])
    ax, ay = O.sie_deflection(x, y, T(1.7), T(1e-10), T(0.0), T(0.0), T(0.0))
    assert torch.allclose(torch.hypot(ax, ay), T([1.7] * 3), atol=1e-6)
    # mean convergence inside rho = theta_E is 1 (Gauss: flux of alpha through the
    # ellipse boundary = 2 * integral of kappa)
    the, q = 1.2, 0.6
    e = (1 - q) / (1 + q)
    n = 4000
    tt = (torch.arange(n, dtype=torch.float64) + 0.5) * 2 * math.pi / n
    # boundary q x^2 + y^2/q = the^2
    xb = the / math.sqrt(q) * torch.cos(tt)
    yb = the * math.sqrt(q) * torch.sin(tt)
    ax, ay = O.sie_deflection(xb, yb, T(the), T(e), T(0.0), T(0.0), T(0.0))
    # outward normal * dl = (dy/dt, -dx/dt) dt
    dxdt = -the / math.sqrt(q) * torch.sin(tt)
    dydt = the * math.sqrt(q) * torch.cos(tt)
    flux = float(((ax * dydt - ay * dxdt) * (2 * math.pi / n)).sum())
    area = math.pi * the * the
    assert abs(flux / (2 * area) - 1.0) < 1e-9


def test_shear_is_gradient_of_its_potential():
    g1, g2 = 0.04, -0.07
    pot = lambda x, y: 0.5 * g1 * (x * x - y * y) + g2 * x * y
    h = 1e-6
    for x, y in [(0.3, -0.2), (1.5, 0.8), (-0.9, 1.1)]:
        ax, ay = O.shear_deflection(T(x), T(y), T(g1), T(g2))
        assert abs(float(ax) - (pot(x + h, y) - pot(x - h, y)) / (2 * h)) < 1e-9
        assert abs(float(ay) - (pot(x, y + h) - pot(x, y - h)) / (2 * h)) < 1e-9


# ---------------------------------------------------------------- NFW (App. A.2)
def F_paper(x):
    """F(x) of App. A.2 at high precision."""
    x = mpmath.mpf(x)
    if x > 1:
        return mpmath.atan(mpmath.sqrt(x * x - 1)) / mpmath.sqrt(x * x - 1)
    if x < 1:
        return mpmath.atanh(mpmath.sqrt(1 - x * x)) / mpmath.sqrt(1 - x * x)
    return mpmath.mpf(1)


def kappa_nfw(X, ks):
    """Eq. (A3): 2 ks (1 - F(X)) / (X^2 - 1), with its limit 2 ks / 3 at X = 1."""
    if abs(X - 1) < 1e-12:
        return 2 * ks / 3
    return float(2 * ks * (1 - F_paper(X)) / (mpmath.mpf(X) ** 2 - 1))


def test_nfw_deflection_matches_radial_integral_of_kappa():
    ks, rs = 0.8, 0.3
    for r in [0.002, 0.05, 0.29, 0.3, 0.31, 0.9, 2.5]:
        # alpha(r) = (2/r) int_0^r kappa(r') r' dr'
        integ = integrate.quad(lambda rp: kappa_nfw(rp / rs, ks) * rp, 0, r,
                               points=[rs] if r > rs else None, epsabs=1e-15, epsrel=1e-12,
                               limit=200)[0]
        ref = 2.0 * integ / r
        ax, ay = O.nfw_deflection(T(r * 0.6), T(r * 0.8), T(ks), T(rs), T(0.0), T(0.0))
        got = math.hypot(float(ax), float(ay))
        assert abs(got - ref) <= 1e-9 * max(abs(ref), 1e-12), (r, got, ref)


def test_nfw_h_against_high_precision():
    mpmath.mp.dps = 40

    def h_ref(x):
        x = mpmath.mpf(x)
        if x < 1:
            return mpmath.log(x / 2) + 2 / mpmath.sqrt(1 - x * x) * mpmath.atanh(mpmath.sqrt((1 - x) / (1 + x)))
        if x > 1:
            return mpmath.log(x / 2) + 2 / mpmath.sqrt(x * x - 1) * mpmath.atan(mpmath.sqrt((x - 1) / (x + 1)))
        return 1 + mpmath.log(mpmath.mpf(1) / 2)

    xs = [1e-9, 1e-6, 5e-4, 1e-3, 0.3, 0.4999999, 0.5000001, 0.999, 0.9995, 0.99999, 1.0,
          1.00001, 1.0005, 1.001, 2.0, 20.0]
    got = O.nfw_h(T(xs))
    for x, g in zip(xs, got):
        ref = float(h_ref(x))
        assert abs(float(g) - ref) <= 1e-11 * abs(ref), (x, float(g), ref)


def test_nfw_poisson_and_truncation():
    ks, rs, xs, ys = 0.5, 0.4, 0.1, -0.2
    fn = lambda x, y: O.nfw_deflection(x, y, T(ks), T(rs), T(xs), T(ys))
    rng = np.random.default_rng(3)
    for _ in range(6):
        x, y = rng.uniform(-1, 1, 2)
        div, curl = _div_curl(fn, x, y, h=1e-5)
        X = math.hypot(x - xs, y - ys) / rs
        assert abs(div - 2 * kappa_nfw(X, ks)) < 1e-6 * max(1.0, kappa_nfw(X, ks))
        assert abs(curl) < 1e-6
    # hard truncation: beyond tau r_s the field is that of a point mass h(tau)
    tau = 2.0
    for r in [0.9, 1.5, 3.0]:
        ax, ay = O.nfw_deflection(T(xs + r), T(ys), T(ks), T(rs), T(xs), T(ys), tau=tau)
        expect = 4 * ks * rs * float(O.nfw_h(T(min(r / rs, tau)))) / (r / rs)
        assert abs(float(ax) - expect) < 1e-12 and abs(float(ay)) < 1e-15


def test_nfw_series_switch_continuity():
    # switch points: x = 1/2 (form for small x) and |v| = 1e-3, v = (1-x)/(1+x)
    for x0 in [0.5, (1 - 1e-3) / (1 + 1e-3), (1 + 1e-3) / (1 - 1e-3)]:
        lo, hi = O.nfw_h(T([x0 * (1 - 1e-13), x0 * (1 + 1e-13)]))
        assert abs(float(hi) - float(lo)) < 1e-12 * abs(float(lo))


# ---------------------------------------------------------------- round lens, lens centre
def _first_order_sie(x, y, the, e1, e2):
    """First order in the ellipticity about the singular isothermal sphere,
    derived by hand from the closed form (q = 1 - 2e, f^2 = 4e, psi = r (1 - 2e
    cos^2 t') to first order, rotated back): with zeta = z/|z| and eps = e1 + i e2,
        alpha/theta_E = zeta - eps conj(zeta)/2 + conj(eps) zeta^3/6 + O(e^2)."""
    z = np.asarray(x) + 1j * np.asarray(y)
    zeta = z / np.abs(z)
    eps = e1 + 1j * e2
    a = the * (zeta - 0.5 * eps * np.conj(zeta) + np.conj(eps) * zeta ** 3 / 6.0)
    return a.real, a.imag


@pytest.mark.parametrize("e", [2e-4, 4e-3])
def test_sie_near_round_lens_matches_first_order_expansion(e):
    """Both evaluations (the series below E_SERIES, the closed form above it)
    leave a residual against the hand-derived first-order expansion that
    shrinks as e^2: a dropped or wrong first-order term would leave O(e)."""
    x = np.array([0.3, -1.2, 0.7, 1.5, -0.4])
    y = np.array([1.1, 0.4, -0.9, -0.2, -1.3])
    res = []
    for scale in (1.0, 0.5):
        ang = 0.7
        e1, e2 = scale * e * math.cos(ang), scale * e * math.sin(ang)
        ax, ay = O.sie_deflection(T(x), T(y), T(1.3), T(e1), T(e2), T(0.0), T(0.0))
        rx, ry = _first_order_sie(x, y, 1.3, e1, e2)
        res.append(max(np.abs(ax.numpy() - rx).max(), np.abs(ay.numpy() - ry).max()))
    assert res[0] < 3.0 * e * e
    assert 3.0 < res[0] / res[1] < 5.0       # O(e^2): halving e quarters the residual


def test_sie_series_and_closed_form_agree_at_the_switch():
    x, y = T([0.3, -1.2, 0.7, 1e-3]), T([1.1, 0.4, -0.9, 2e-3])
    for ang in (0.3, 2.0, -1.1):
        lo = O.sie_deflection(x, y, T(1.2), T(O.E_SERIES * (1 - 1e-9) * math.cos(ang)),
                              T(O.E_SERIES * (1 - 1e-9) * math.sin(ang)), T(0.01), T(-0.02))
        hi = O.sie_deflection(x, y, T(1.2), T(O.E_SERIES * (1 + 1e-9) * math.cos(ang)),
                              T(O.E_SERIES * (1 + 1e-9) * math.sin(ang)), T(0.01), T(-0.02))
        for a, b in zip(lo, hi):
            assert float((a - b).abs().max()) < 1e-11


def test_sie_series_matches_schramm_integral_for_a_nearly_round_lens():
    e = 2e-4
    q = (1 - e) / (1 + e)
    for x, y in [(0.4, 1.1), (-1.3, 0.2), (0.05, -0.7)]:
        ax, ay = O.sie_deflection(T(x), T(y), T(1.1), T(e), T(0.0), T(0.0), T(0.0))
        rx, ry = schramm_alpha(x, y, 1.1, q)
        assert abs(float(ax) - rx) < 1e-10 and abs(float(ay) - ry) < 1e-10


def test_round_lens_gradient_is_finite_and_matches_central_differences():
    """At e1 = e2 = 0 the position angle is undefined, but the deflection is
    smooth in (e1, e2): the gradient exists and equals central differences
    (which straddle e = 0)."""
    x, y = T([0.3, -1.2, 0.7, 1e-3]), T([1.1, 0.4, -0.9, 2e-3])
    wx, wy = T([1.0, 2.0, 3.0, 4.0]), T([-1.0, 0.5, 2.0, 1.0])

    def f(p):
        ax, ay = O.sie_deflection(x, y, p[0], p[1], p[2], p[3], p[4])
        return (ax * wx + ay * wy).sum()

    p = T([1.2, 0.0, 0.0, 0.01, -0.02]).requires_grad_(True)
    (g,) = torch.autograd.grad(f(p), p)
    assert bool(torch.isfinite(g).all())
    h = 1e-6
    for i in range(5):
        pp, pm = p.detach().clone(), p.detach().clone()
        pp[i] += h
        pm[i] -= h
        fd = (float(f(pp)) - float(f(pm))) / (2 * h)
        assert abs(float(g[i]) - fd) < 1e-7 * max(1.0, abs(fd)), (i, float(g[i]), fd)


def test_lens_equation_sign_on_the_einstein_ring():
    """beta = theta - alpha: for a singular isothermal sphere a ray on the
    Einstein ring maps to the source-plane origin, and a ray at 2 theta_E to
    theta_E along the same direction."""
    the = 1.3
    lens = T([the, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    ang = torch.linspace(0, 2 * math.pi, 9, dtype=torch.float64)[:-1]
    for rad, expect in ((the, 0.0), (2 * the, the)):
        bx, by = O.ray_shoot(rad * torch.cos(ang), rad * torch.sin(ang), lens)
        assert torch.allclose(bx, expect * torch.cos(ang), atol=1e-13)
        assert torch.allclose(by, expect * torch.sin(ang), atol=1e-13)
    # off-centre lens: the same about its centre
    lens = T([the, 0.1, -0.05, 0.2, -0.3, 0.0, 0.0])
    bx, by = O.ray_shoot(T([0.2]), T([-0.3]), lens)
    assert float(bx) == 0.2 and float(by) == -0.3     # the centre ray is not deflected


def test_rays_on_the_lens_or_subhalo_centre_are_not_deflected():
    lens = T([1.1, 0.12, -0.07, 0.05, -0.04, 0.0, 0.0, 0.4, 0.2, 0.3, 0.25]).requires_grad_(True)
    x, y = T([0.05, 0.3, 0.9]), T([-0.04, 0.25, 0.1])
    ax, ay = O.deflection(x, y, lens, n_sub=1)
    # ray 0 sits on the SIE centre, ray 1 on the subhalo centre
    ax_sie, ay_sie = O.sie_deflection(x, y, lens[0], lens[1], lens[2], lens[3], lens[4])
    nx, ny = O.nfw_deflection(x, y, lens[7], lens[8], lens[9], lens[10])
    assert float(ax_sie[0].detach()) == 0.0 and float(ay_sie[0].detach()) == 0.0
    assert float(nx[1].detach()) == 0.0 and float(ny[1].detach()) == 0.0
    (g,) = torch.autograd.grad((ax + ay).sum(), lens)
    assert bool(torch.isfinite(g).all())
