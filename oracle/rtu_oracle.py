"""FP64 CPU oracle of the RTU-grid lens likelihood and its gradient.

TEST INFRASTRUCTURE ONLY.  Tests, the smoke check and the CPU-baseline leg of
the benchmark call this module; the GPU library never does, and this module
imports nothing from the GPU package.  It is written for a reader to check by
eye against the paper (Enzi et al., "Gaussian processes on ray-guided
transformed uniform grids"): plain float64 tensor operations in the order the
paper gives them, library primitives (sort, FFT, conv2d) as single steps, and
the gradient as reverse-mode differentiation of this forward definition (the
paper's model is differentiated the same way, by automatic differentiation).

Where the paper is silent or ambiguous, the reading taken is stated at the
function that implements it.  Status bits follow the GPU library's contract:
1 non-finite result, 2 non-monotone smoothed CDF (slopes clamped),
4 fewer masked pixels than nodes + 1, 8 parameter outside its domain.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np
import torch

DT = torch.float64
S0 = 0.01            # softplus scale s_0 (Sec. 2.1, eq. 3)
K_NODES = 22         # Chebyshev nodes = degree 21 + 1 (App. C, step iii; Fig. C1)
N_LENS_BASE = 7
N_PER_SUB = 4
N_PER_GAUSS = 6      # lens-light Gaussian: A, sigma, e1, e2, x_c, y_c

ST_NONFINITE = 1
ST_NONMONOTONE = 2
ST_MASK_SMALL = 4
ST_DOMAIN = 8


def _t(a) -> torch.Tensor:
    return torch.as_tensor(np.asarray(a), dtype=DT)


# ------------------------------------------------------------------ image plane
def pixel_centres(n_img: int, pix: float):
    """Pixel (i, j) centre: theta = ((j - (N-1)/2) pix, (i - (N-1)/2) pix);
    row i <-> y, column j <-> x.  Returns x, y of shape [N*N] (row-major)."""
    c = (torch.arange(n_img, dtype=DT) - 0.5 * (n_img - 1)) * pix
    y, x = torch.meshgrid(c, c, indexing="ij")
    return x.reshape(-1), y.reshape(-1)


def subray_positions(n_img: int, pix: float, ss: int):
    """Sub-ray (a, b) of pixel p sits at the pixel centre plus
    (((b + 1/2)/ss - 1/2) pix, ((a + 1/2)/ss - 1/2) pix)  (Sec. 2.3 sub-sampling;
    a regular ss x ss lattice centred in the pixel).  Shape [N*N, ss*ss]."""
    xc, yc = pixel_centres(n_img, pix)
    off = ((torch.arange(ss, dtype=DT) + 0.5) / ss - 0.5) * pix
    oy, ox = torch.meshgrid(off, off, indexing="ij")
    return xc[:, None] + ox.reshape(1, -1), yc[:, None] + oy.reshape(1, -1)


# ------------------------------------------------------------------ lens mass
def q_phi_from_e(e1, e2):
    """Ellipticity components -> axis ratio and angle:
    e = |(e1, e2)|, q = (1 - e)/(1 + e), phi = atan2(e2, e1)/2 (App. A.1 infers
    ellipticities; this is the usual convention)."""
    e = torch.sqrt(e1 * e1 + e2 * e2)
    return (1.0 - e) / (1.0 + e), 0.5 * torch.atan2(e2, e1), e


E_SERIES = 1e-3     # below this |(e1, e2)| the SIE is summed as its series about the SIS


def sie_deflection(x, y, theta_e, e1, e2, x0, y0):
    """Deflection of the EPL of App. A.1, eq. (A1), at slope gamma = 2 (singular
    isothermal ellipsoid): kappa = (theta_E / 2) / rho, rho^2 = q x'^2 + y'^2 / q in
    the frame rotated by phi about (x0, y0).  Closed form with f = sqrt(1 - q^2),
    psi = sqrt(q^2 x'^2 + y'^2):
        a'_x = theta_E sqrt(q)/f atan(f x'/psi),  a'_y = theta_E sqrt(q)/f atanh(f y'/psi),
    rotated back by phi.

    For a nearly round lens (|e| < E_SERIES) the position angle is ill defined
    and the closed form divides by f -> 0; there the same deflection is written
    without any angle.  With complex positions z = (x - x0) + i (y - y0) and
    ellipticity eps = e1 + i e2, the frame change and the elliptical angle
    combine into u = m/|m|, m = z - eps conj(z), and the deflection is
        alpha = theta_E sqrt(1 - |eps|^2) u G(conj(eps) u^2),
        G(w) = atan(sqrt w)/sqrt w = sum_k (-w)^k / (2k + 1)
    (the hypergeometric form of the elliptical power law of Tessore & Metcalf
    2015 at slope 2, with e^{2 i phi} absorbed into eps), summed as its series
    (|w| = |eps| < E_SERIES: eight terms reach 1e-24).  At eps = 0 it is the
    singular isothermal sphere theta_E z/|z|, and it is smooth in (e1, e2).

    A ray exactly on the lens centre (psi = 0), where the direction of the
    deflection is undefined, is not deflected (alpha = 0, the value the
    symmetric limit averages to)."""
    dx, dy = x - x0, y - y0
    centre = (dx == 0) & (dy == 0)
    # stand-in position for rays on the centre: keeps every branch finite
    dx = torch.where(centre, torch.ones_like(dx), dx)
    dy = torch.where(centre, torch.zeros_like(dy), dy)
    if float(torch.hypot(e1.detach(), e2.detach())) >= E_SERIES:
        q, phi, e = q_phi_from_e(e1, e2)
        c, s = torch.cos(phi), torch.sin(phi)
        xp = c * dx + s * dy
        yp = -s * dx + c * dy
        f = 2.0 * torch.sqrt(e) / (1.0 + e)          # = sqrt(1 - q^2) without cancellation
        psi = torch.sqrt(q * q * xp * xp + yp * yp)
        pref = theta_e * torch.sqrt(q) / f
        axp = pref * torch.atan(f * xp / psi)
        ayp = pref * torch.atanh(f * yp / psi)
        ax, ay = c * axp - s * ayp, s * axp + c * ayp
    else:
        z = torch.complex(dx, dy)
        eps = torch.complex(e1 * torch.ones_like(dx), e2 * torch.ones_like(dx))
        m = z - eps * z.conj()
        u = m / m.abs()
        w = eps.conj() * u * u
        G = sum((-w) ** k / (2 * k + 1) for k in range(8))
        a = theta_e * torch.sqrt(1.0 - (e1 * e1 + e2 * e2)) * u * G
        ax, ay = a.real, a.imag
    zero = torch.zeros_like(ax)
    return torch.where(centre, zero, ax), torch.where(centre, zero, ay)


def epl_deflection(x, y, theta_e, e1, e2, x0, y0, gamma, tol=1e-17):
    """Deflection of the elliptical power law of App. A.1, eq. (A1):
    kappa = (3 - gamma)/2 (theta_E / rho)^(gamma - 1), rho^2 = q x'^2 + y'^2/q.
    Tessore & Metcalf (2015) give it in the lens frame as a hypergeometric
    function of the elliptical angle.  With complex z = (x - x0) + i (y - y0),
    eps = e1 + i e2, m = z - eps conj(z), u = m/|m| and t = gamma - 1 (the
    frame change absorbed into eps as in sie_deflection) it reads
        alpha = Lam^t |m|^(1 - t) u F(-conj(eps) u^2),  Lam = theta_E sqrt(1 - |eps|^2),
        F(w) = 2F1(1, t/2; 2 - t/2; w) = sum_n c_n w^n,
        c_0 = 1,  c_n = c_{n-1} (2n - 2 + t) / (2n + 2 - t),
    the series summed until c_n |eps|^n < tol (|w| = |eps| < 1).  At gamma = 2
    it is sie_deflection; it has no angle and is smooth in (e1, e2).  A ray on
    the centre is not deflected."""
    t = gamma - 1.0
    dx, dy = x - x0, y - y0
    centre = (dx == 0) & (dy == 0)
    dx = torch.where(centre, torch.ones_like(dx), dx)
    dy = torch.where(centre, torch.zeros_like(dy), dy)
    z = torch.complex(dx, dy)
    eps = torch.complex(e1 * torch.ones_like(dx), e2 * torch.ones_like(dx))
    m = z - eps * z.conj()
    am = m.abs()
    u = m / am
    w = -eps.conj() * u * u
    e = float(torch.hypot(e1.detach(), e2.detach()))
    F = torch.zeros_like(w)
    c = torch.ones((), dtype=DT) + 0.0 * t
    wn = torch.ones_like(w)
    n = 0
    while True:
        F = F + c * wn
        n += 1
        c = c * (2.0 * n - 2.0 + t) / (2.0 * n + 2.0 - t)
        wn = wn * w
        if float(c.detach()) * e ** n < tol or n > 5000:
            break
    lam = theta_e * torch.sqrt(1.0 - (e1 * e1 + e2 * e2))
    a = lam ** t * am ** (1.0 - t) * u * F
    zero = torch.zeros_like(dx)
    return torch.where(centre, zero, a.real), torch.where(centre, zero, a.imag)


def shear_deflection(x, y, g1, g2):
    """External shear about the origin, potential (g1 (x^2 - y^2) + 2 g2 x y)/2."""
    return g1 * x + g2 * y, g2 * x - g1 * y


def _nfw_T(v):
    """T(v) = atanh(sqrt v)/sqrt v for v > 0, atan(sqrt(-v))/sqrt(-v) for v < 0,
    T(0) = 1; the power series 1 + v/3 + v^2/5 + ... near v = 0."""
    small = v.abs() < 1e-3
    vs = torch.where(small, torch.full_like(v, 0.5), v)
    pos = vs > 0
    sp = torch.sqrt(torch.where(pos, vs, torch.ones_like(vs)))
    sn = torch.sqrt(torch.where(pos, torch.ones_like(vs), -vs))
    direct = torch.where(pos, torch.atanh(sp) / sp, torch.atan(sn) / sn)
    series = 1.0 + v / 3.0 + v * v / 5.0 + v ** 3 / 7.0 + v ** 4 / 9.0
    return torch.where(small, series, direct)


def nfw_h(x):
    """Projected-mass function of the NFW profile (App. A.2, eqs. A2-A3):
    h(x) = ln(x/2) + 2/sqrt(1-x^2) atanh(sqrt((1-x)/(1+x))) for x < 1,
           ln(x/2) + 2/sqrt(x^2-1) atan(sqrt((x-1)/(x+1)))  for x > 1.
    For x >= 1/2 it is evaluated as ln(x/2) + 2 T(v)/(1+x), v = (1-x)/(1+x), which
    covers both branches and gives h(1) = 1 + ln 1/2.  Below x = 1/2 the two
    logarithms cancel; there the same function is written, with c = sqrt(1-x^2)
    and using 2 atanh(sqrt((1-x)/(1+x))) = ln((1+c)/x), as
        h = ln(2/x) x^2 / ((1+c) c) + log1p(-x^2 / (2(1+c))) / c."""
    lo = x < 0.5
    xl = torch.where(lo, x, torch.full_like(x, 0.25))
    c = torch.sqrt(1.0 - xl * xl)
    h_lo = torch.log(2.0 / xl) * xl * xl / ((1.0 + c) * c) + torch.log1p(-xl * xl / (2.0 * (1.0 + c))) / c
    xh = torch.where(lo, torch.ones_like(x), x)
    v = (1.0 - xh) / (1.0 + xh)
    h_hi = torch.log(0.5 * xh) + 2.0 * _nfw_T(v) / (1.0 + xh)
    return torch.where(lo, h_lo, h_hi)


def nfw_deflection(x, y, ks, rs, xs, ys, tau: float = 0.0):
    """Radial deflection of the projected NFW of eq. (A3):
    alpha = 4 kappa_s r_s h(X)/X along d/|d|, d = theta - centre, X = |d|/r_s.
    With tau > 0 the projected mass is frozen beyond X = tau (hard truncation:
    h(min(X, tau)))."""
    dx, dy = x - xs, y - ys
    centre = (dx == 0) & (dy == 0)       # a ray on the subhalo centre is not deflected
    dx = torch.where(centre, torch.ones_like(dx), dx)
    r = torch.sqrt(dx * dx + dy * dy)
    X = r / rs
    Xh = torch.clamp(X, max=tau) if tau > 0 else X
    # alpha_vec = 4 ks rs h(X)/X * d/|d| = 4 ks rs^2 h(X) d / r^2
    fac = 4.0 * ks * rs * nfw_h(Xh) / (X * r)
    fac = torch.where(centre, torch.zeros_like(fac), fac)
    return fac * dx, fac * dy


def lens_base(epl: bool = False) -> int:
    """Lens parameters before the subhaloes: theta_E, e1, e2, x0, y0, gamma1,
    gamma2, and with the EPL its slope gamma."""
    return N_LENS_BASE + (1 if epl else 0)


def deflection(x, y, lens, n_sub: int = 0, tau: float = 0.0, epl: bool = False):
    """Total deflection: SIE (or with epl the EPL, slope lens[7]) + external
    shear + n_sub NFW subhaloes."""
    if epl:
        ax, ay = epl_deflection(x, y, lens[0], lens[1], lens[2], lens[3], lens[4], lens[7])
    else:
        ax, ay = sie_deflection(x, y, lens[0], lens[1], lens[2], lens[3], lens[4])
    sx, sy = shear_deflection(x, y, lens[5], lens[6])
    ax, ay = ax + sx, ay + sy
    for j in range(n_sub):
        b = lens_base(epl) + N_PER_SUB * j
        nx, ny = nfw_deflection(x, y, lens[b], lens[b + 1], lens[b + 2], lens[b + 3], tau)
        ax, ay = ax + nx, ay + ny
    return ax, ay


def ray_shoot(x, y, lens, n_sub=0, tau=0.0, epl=False):
    """Lens equation beta = theta - alpha(theta)."""
    ax, ay = deflection(x, y, lens, n_sub, tau, epl)
    return x - ax, y - ay


# ------------------------------------------------------------------ lens light
def mge_light(x, y, light):
    """Lens light as a multi-Gaussian expansion (App. A, Multi Gaussian
    Expansion): component n, with parameters (A_n, sigma_n, e1_n, e2_n, x_n, y_n),
    adds A_n/(2 pi) exp(-rho_n^2/(2 sigma_n^2)), where rho_n^2 = q_n x'^2 + y'^2/q_n
    in the frame centred on (x_n, y_n) and rotated by the component's position
    angle.  The paper frees q_n and the angle per component and parametrises
    ellipticities as for the mass; q_n and the angle come from (e1_n, e2_n) with
    q_phi_from_e (reading: the mass's convention).  The light is not lensed: it
    is evaluated at the image-plane positions.  Through the angle this form is
    not differentiable at e_n = 0 exactly."""
    total = torch.zeros_like(x)
    for n in range(light.shape[0] // N_PER_GAUSS):
        A, sig, e1, e2, xc, yc = (light[N_PER_GAUSS * n + k] for k in range(N_PER_GAUSS))
        q, phi, _ = q_phi_from_e(e1, e2)
        c, s = torch.cos(phi), torch.sin(phi)
        dx, dy = x - xc, y - yc
        xp = c * dx + s * dy
        yp = -s * dx + c * dy
        rho2 = q * xp * xp + yp * yp / q
        total = total + A / (2.0 * math.pi) * torch.exp(-0.5 * rho2 / (sig * sig))
    return total


# ------------------------------------------------------------------ RTU transform
def chebyshev_nodes(K: int = K_NODES):
    """Chebyshev nodes mapped to (0, 1): u_k = (1 - cos((2k - 1) pi / (2K)))/2."""
    k = torch.arange(1, K + 1, dtype=DT)
    return 0.5 * (1.0 - torch.cos((2.0 * k - 1.0) * math.pi / (2.0 * K)))


def standardise(bx, by, w=None):
    """App. C step (i): subtract the mean per axis and divide by the smaller of
    the two (population) standard deviations.  With ray weights w (Sec. 6.3)
    the moments are weighted (a ray of integer weight k counts as k rays)."""
    if w is None:
        mx, my = bx.mean(), by.mean()
        sx = torch.sqrt(((bx - mx) ** 2).mean())
        sy = torch.sqrt(((by - my) ** 2).mean())
    else:
        W = w.sum()
        mx, my = (w * bx).sum() / W, (w * by).sum() / W
        sx = torch.sqrt((w * (bx - mx) ** 2).sum() / W)
        sy = torch.sqrt((w * (by - my) ** 2).sum() / W)
    s = torch.minimum(sx, sy)
    return mx, my, s


def quantiles_type7(z, u, picks=None):
    """App. C step (ii): the eCDF by sorting, and its inverse between the sorted
    positions by linear interpolation (Sec. 2.2, App. C first paragraph):
    h = (M-1) u, j = floor h, Q(u) = (1 - (h-j)) z_(j) + (h-j) z_(j+1).
    Ties are ordered by ray index (stable sort).  Returns Q and the sorted
    positions' original indices at j and j+1.

    picks = (i0, i1), ray indices standing in for the order statistics at j and
    j + 1: where two rays are closer than the rounding of an evaluation,
    another evaluation may order them the other way; with its picks the same
    formula gives the quantiles and their derivatives for that order."""
    M = z.shape[0]
    h = (M - 1) * u
    j = torch.floor(h).long()
    t = h - j.to(DT)
    if picks is not None:
        i0, i1 = (torch.as_tensor(np.asarray(p), dtype=torch.long) for p in picks)
        return (1.0 - t) * z[i0] + t * z[i1], i0, i1
    zs, order = torch.sort(z, stable=True)
    j1 = torch.clamp(j + 1, max=M - 1)
    q = (1.0 - t) * zs[j] + t * zs[j1]
    return q, order[j], order[j1]


def quantiles_weighted(z, w, u, picks=None):
    """Quantiles of rays with weights (Sec. 6.3, the weighted RTU grid).
    Reading: a weight counts rays, so that a ray of integer weight k stands for
    k copies of itself: in sorted order (ties by ray index) ray i holds the
    cumulative-weight interval [C_{i-1}, C_i), E(r) is the ray holding
    position r, and with h = (W - 1) u, W = sum w, j = floor h,
        Q(u) = (1 - (h - j)) z_E(j) + (h - j) z_E(j+1),
    E clamped to the last ray.  Unit weights give type 7 (quantiles_type7);
    rays of weight 0 are never picked.  picks as for quantiles_type7."""
    W = w.sum()
    h = (W - 1.0) * u
    j = torch.floor(h)
    t = h - j
    if picks is not None:
        i0, i1 = (torch.as_tensor(np.asarray(p), dtype=torch.long) for p in picks)
        return (1.0 - t) * z[i0] + t * z[i1], i0, i1
    zs, order = torch.sort(z, stable=True)
    C = torch.cumsum(w[order], 0)
    M = z.shape[0]
    e0 = torch.clamp(torch.searchsorted(C, j, right=True), max=M - 1)
    e1 = torch.clamp(torch.searchsorted(C, j + 1.0, right=True), max=M - 1)
    return (1.0 - t) * zs[e0] + t * zs[e1], order[e0], order[e1]


def chebyshev_T_U(tn, D: int):
    """T_0..T_D and U_0..U_D at points tn by their three-term recurrences."""
    T = [torch.ones_like(tn), tn]
    U = [torch.ones_like(tn), 2.0 * tn]
    for _ in range(2, D + 1):
        T.append(2.0 * tn * T[-1] - T[-2])
        U.append(2.0 * tn * U[-1] - U[-2])
    return torch.stack(T[:D + 1]), torch.stack(U[:D + 1])


def qf_polynomial(q, u):
    """App. C step (iii): polynomial of degree K-1 (21 for K = 22) through the
    quantile function at the K Chebyshev nodes.  With as many nodes as
    coefficients the weighted fit interpolates the nodes exactly, so the node
    weights do not change it.  In t = 2u - 1:
        c_j = (2 - delta_j0)/K sum_k q_k T_j(t_k),
        p'(u) = dp/du = 2 sum_j j c_j U_{j-1}(t).
    Returns the slope p'(u_k) at every node."""
    K = q.shape[0]
    tn = 2.0 * u - 1.0
    T, U = chebyshev_T_U(tn, K - 1)
    c = (T @ q) * (2.0 / K)
    c = torch.cat([c[:1] * 0.5, c[1:]])
    j = torch.arange(1, K, dtype=DT)
    dp = 2.0 * ((j[:, None] * c[1:, None]) * U[:K - 1]).sum(0)
    return dp


def cdf_spline(z, X, S, u):
    """App. C step (iv): the smoothed CDF as the cubic Hermite spline through
    (X_k, u_k) with slopes S_k = 1/p'(u_k); linear continuation with the end
    slopes outside [X_1, X_K].  The interval of z is the largest k with
    X_k <= z (so zero-width intervals are never used)."""
    K = X.shape[0]
    k = torch.searchsorted(X.detach().contiguous(), z.detach().contiguous(), right=True)  # #knots <= z
    inner = (k >= 1) & (k <= K - 1)
    kl = torch.clamp(k - 1, 0, K - 2)
    Xl, Xr = X[kl], X[kl + 1]
    h = torch.where(inner, Xr - Xl, torch.ones_like(Xl))
    t = (z - Xl) / h
    t2, t3 = t * t, t * t * t
    h00 = 2 * t3 - 3 * t2 + 1
    h10 = t3 - 2 * t2 + t
    h01 = -2 * t3 + 3 * t2
    h11 = t3 - t2
    g_in = h00 * u[kl] + h10 * h * S[kl] + h01 * u[kl + 1] + h11 * h * S[kl + 1]
    g_lo = u[0] + S[0] * (z - X[0])
    g_hi = u[K - 1] + S[K - 1] * (z - X[K - 1])
    return torch.where(k == 0, g_lo, torch.where(k >= K, g_hi, g_in))


def build_transform(bxm, bym, K: int = K_NODES, picks=None, weights=None):
    """RTU transform from the masked rays (Sec. 2.2; App. C steps i-iv).
    Returns a dict with mu, s, knots X[2][K], slopes S[2][K], nodes u, the
    selected ray indices and the status bits.  picks (optional, per axis the
    pair (i0, i1) of quantiles_type7) fixes which rays stand for the order
    statistics.  weights (optional, per masked ray): the weighted RTU grid of
    Sec. 6.3 (quantiles_weighted, weighted standardisation)."""
    u = chebyshev_nodes(K)
    mx, my, s = standardise(bxm, bym, weights)
    out = {"u": u, "mu": (mx, my), "s": s, "status": 0}
    X, S, idx = [], [], []
    for ax, zc in enumerate(((bxm - mx) / s, (bym - my) / s)):
        pk = None if picks is None else picks[ax]
        q, i0, i1 = quantiles_type7(zc, u, pk) if weights is None else quantiles_weighted(zc, weights, u, pk)
        dp = qf_polynomial(q, u)
        # X_k = p(u_k) equals q_k exactly (interpolation); q_k is used directly.
        eps = 1e-6 * (q[-1] - q[0]).detach()
        bad = bool((dp.detach() <= eps).any()) or bool((q[1:] <= q[:-1]).any())
        if bad:
            out["status"] |= ST_NONMONOTONE
        dp = torch.where(dp > eps, dp, eps.expand_as(dp))
        X.append(q)
        S.append(1.0 / dp)
        idx.append((i0, i1))
    out["X"], out["S"], out["idx"] = X, S, idx
    return out


def uniform_box_of(bxm, bym, picks=None):
    """Sec. 2.1: the extent of the uniform grid, the smallest square box that
    holds the masked rays.  Reading: the side L is the larger of the two
    coordinate ranges (the x range on a tie), and the box is centred on the
    rays' bounding box along both axes (along the longer axis it then spans the
    range exactly).  The extremes are the order statistics of rank 0 and M - 1
    (the type-7 quantiles at u = 0 and 1, ties by ray index) and are
    differentiated as selections.  picks = per axis (index of the minimum,
    index of the maximum) fixes which rays stand for them.  Fewer than two
    masked rays, or a zero range on both axes: status bit 4 and the box of
    side 1 at the rays' minimum (or at 0)."""
    status = 0
    M = bxm.shape[0]
    ends = torch.tensor([0.0, 1.0], dtype=DT)
    lo_hi, idx = [], []
    for ax, z in enumerate((bxm, bym)):
        if M == 0:
            lo_hi.append((torch.zeros((), dtype=DT), torch.zeros((), dtype=DT)))
            idx.append((torch.zeros(1, dtype=torch.long), torch.zeros(1, dtype=torch.long)))
            continue
        pk = None if picks is None else ([picks[ax][0], picks[ax][1]], [picks[ax][0], picks[ax][1]])
        q, i0, _ = quantiles_type7(z, ends, pk)
        lo_hi.append((q[0], q[1]))
        idx.append((i0[:1], i0[1:]))
    rx = lo_hi[0][1] - lo_hi[0][0]
    ry = lo_hi[1][1] - lo_hi[1][0]
    side = torch.where(rx >= ry, rx, ry)
    if M < 2 or not bool(side > 0):
        status |= ST_MASK_SMALL
        return {"lo": (lo_hi[0][0].detach(), lo_hi[1][0].detach()), "side": torch.ones((), dtype=DT),
                "idx": idx, "status": status}
    lo = tuple(0.5 * (a + b) - 0.5 * side for a, b in lo_hi)
    return {"lo": lo, "side": side, "idx": idx, "status": status}


def rtu_transform(bx, by, tr):
    """Eq. (5): y = g(x) = (CDF_1(x_1), CDF_2(x_2)) on standardised coordinates."""
    zx = (bx - tr["mu"][0]) / tr["s"]
    zy = (by - tr["mu"][1]) / tr["s"]
    return (cdf_spline(zx, tr["X"][0], tr["S"][0], tr["u"]),
            cdf_spline(zy, tr["X"][1], tr["S"][1], tr["u"]))


# ------------------------------------------------------------------ GP source
def fft_freqs(n: int):
    """Signed integer FFT frequencies (cycles per unit-square side)."""
    k = torch.arange(n, dtype=DT)
    return torch.where(k < n / 2, k, k - n)


def matern_sqrtP(n: int, ps):
    """Square root of the Matern spectrum of eq. (4) on the n x n FFT grid:
    P(k) = sigma^2 4 pi n_s (2 n_s/zeta^2)^n_s (2 n_s/zeta^2 + k^2)^-(n_s + 1)."""
    sig, ns, zeta = ps[0], ps[1], ps[2]
    fk = fft_freqs(n)
    k2 = fk[:, None] ** 2 + fk[None, :] ** 2
    a = 2.0 * ns / (zeta * zeta)
    P = sig * sig * 4.0 * math.pi * ns * a ** ns * (a + k2) ** (-(ns + 1.0))
    return torch.sqrt(P)


def softplus(x):
    """Eq. (2), log(1 + e^x), evaluated as max(x, 0) + log1p(e^-|x|)."""
    return torch.clamp(x, min=0.0) + torch.log1p(torch.exp(-x.abs()))


def gp_field(w, sqrtP):
    """Eq. (1): f = Re IDFT(sqrt(P) * DFT(w)), forward DFT unnormalised and the
    inverse divided by n^2.  The latent is the real white-noise field w."""
    F = torch.fft.fft2(w.to(torch.complex128))
    return torch.fft.ifft2(sqrtP * F).real


def positive_source(f, alpha):
    """Eqs. (2)-(3): s = (s0 softplus(f/s0))^alpha_src."""
    return (S0 * softplus(f / S0)) ** alpha


def gp_source(w, ps):
    """Source grid from the latent and the spectrum parameters, eqs. (1)-(4)."""
    f = gp_field(w, matern_sqrtP(w.shape[0], ps))
    return positive_source(f, ps[3]), f


def bilinear(s, yx, yy, cell_shift: float = 0.0):
    """Bilinear interpolation of the grid s (Sec. 2.1) at unit-square positions.
    Node (i, j) sits at ((j + 1/2)/n, (i + 1/2)/n); values outside the grid are
    zero.  The cell of a position t (in node units) is floor(t + cell_shift);
    the interpolant is continuous, so a small shift changes only which side's
    derivative a position on a cell edge takes."""
    n = s.shape[0]
    tx = yx * n - 0.5
    ty = yy * n - 0.5
    j0 = torch.floor(tx.detach() + cell_shift)
    i0 = torch.floor(ty.detach() + cell_shift)
    fx = tx - j0
    fy = ty - i0
    j0 = j0.long()
    i0 = i0.long()
    sflat = s.reshape(-1)

    def at(i, j):
        ok = (i >= 0) & (i < n) & (j >= 0) & (j < n)
        ii = torch.where(ok, i * n + j, torch.zeros_like(i))
        return torch.where(ok, sflat[ii], torch.zeros_like(fx))

    return ((1 - fx) * (1 - fy) * at(i0, j0) + fx * (1 - fy) * at(i0, j0 + 1)
            + (1 - fx) * fy * at(i0 + 1, j0) + fx * fy * at(i0 + 1, j0 + 1))


# ------------------------------------------------------------------ image and loss
def psf_convolve(u, psf):
    """Zero-padded 'same' convolution of the image with the PSF (kernel flipped,
    not renormalised)."""
    k = psf.shape[0]
    kern = torch.flip(psf, dims=(0, 1))[None, None]
    return torch.nn.functional.conv2d(u[None, None], kern, padding=k // 2)[0, 0]


def forward(lens, ps, w, obs, n_sub=0, tau=0.0, uniform_box=None, return_all=False, cell_shift=0.0,
            round32=False, picks=None):
    """One evaluation of the lens model.

    obs: dict with n_img, pix, ss, image[N,N], sigma[N,N], psf[K,K], mask[N,N],
    and optionally n_gauss: the last N_PER_GAUSS n_gauss entries of lens are
    lens-light Gaussians (mge_light), added to every sub-ray's value before the
    sub-ray mean and the PSF; grid = "uniform": the source grid spans the
    smallest square box of the masked rays (Sec. 2.1, uniform_box_of) instead
    of the RTU transform; ray_weights[N,N]: per-pixel weights of the masked
    rays for the weighted RTU grid (Sec. 6.3, quantiles_weighted);
    lens_model = "epl": the main deflector is the EPL with its slope as lens
    parameter 7 (epl_deflection), the subhaloes following it.
    uniform_box: if given as (x_lo, y_lo, side), the RTU transform is replaced by
    the plain affine map of that box onto the unit square (the paper's uniform
    grid, Sec. 2.1).
    round32: round the ray positions, the knots and slopes and the grid
    positions to binary32 (a model of an evaluation that shoots rays and
    evaluates the spline in binary32 with the quantile fit in binary64).
    picks: the masked rays standing for the order statistics (build_transform)."""
    N, pix, ss = obs["n_img"], obs["pix"], obs["ss"]
    epl = obs.get("lens_model", "sie") == "epl"
    r32 = (lambda t: t.float().to(DT)) if round32 else (lambda t: t)
    status = 0
    lv, pv = lens.detach(), ps.detach()
    n_gauss = int(obs.get("n_gauss", 0))
    light = lens[lens.shape[0] - N_PER_GAUSS * n_gauss:] if n_gauss else None
    if float(lv[0]) <= 0 or float(torch.hypot(lv[1], lv[2])) >= 1 or \
            any(float(lv[lens_base(epl) + N_PER_SUB * j + 1]) <= 0 for j in range(n_sub)) or \
            (epl and not (1.0 < float(lv[7]) < 3.0)) or \
            bool((pv[:3] <= 0).any()) or bool((obs["sigma"] <= 0).any()):
        status |= ST_DOMAIN
    if n_gauss:
        lt = light.detach().reshape(n_gauss, N_PER_GAUSS)
        if bool((lt[:, 1] <= 0).any()) or bool((torch.hypot(lt[:, 2], lt[:, 3]) >= 1).any()):
            status |= ST_DOMAIN
    xr, yr = subray_positions(N, pix, ss)
    bx, by = ray_shoot(xr, yr, lens, n_sub, tau, epl)
    bx, by = r32(bx), r32(by)
    mflat = obs["mask"].reshape(-1).bool()
    xc, yc = pixel_centres(N, pix)
    M = int(mflat.sum())
    uniform = obs.get("grid", "rtu") == "uniform"
    if M < (2 if uniform else K_NODES + 1):
        status |= ST_MASK_SMALL
    tr = None
    if uniform:
        bxm, bym = ray_shoot(xc[mflat], yc[mflat], lens, n_sub, tau, epl)
        tr = uniform_box_of(r32(bxm), r32(bym), picks=picks)
        status |= tr["status"]
        gx, gy = (bx - tr["lo"][0]) / tr["side"], (by - tr["lo"][1]) / tr["side"]
        gx, gy = r32(gx), r32(gy)
    elif uniform_box is None:
        bxm, bym = ray_shoot(xc[mflat], yc[mflat], lens, n_sub, tau, epl)
        rw = obs.get("ray_weights")
        rw = None if rw is None else _t(rw).reshape(-1)[mflat]
        tr = build_transform(r32(bxm), r32(bym), picks=picks, weights=rw)
        status |= tr["status"]
        if round32:
            tr["X"] = [r32(x) for x in tr["X"]]
            tr["S"] = [r32(x) for x in tr["S"]]
        gx, gy = rtu_transform(bx, by, tr)
        gx, gy = r32(gx), r32(gy)
    else:
        x_lo, y_lo, side = uniform_box
        gx, gy = (bx - x_lo) / side, (by - y_lo) / side
    s_grid, f = gp_source(w, ps)
    v = bilinear(s_grid, gx, gy, cell_shift)
    if n_gauss:
        v = v + mge_light(xr, yr, light)
    u_img = v.mean(dim=1).reshape(N, N)
    m = psf_convolve(u_img, obs["psf"])
    res = (m - obs["image"]) / obs["sigma"]
    chi2 = (res ** 2).sum()
    loss = 0.5 * chi2 + 0.5 * (w ** 2).sum()
    chi2_mask = (res.reshape(-1)[mflat] ** 2).mean() if M > 0 else torch.zeros((), dtype=DT)
    if not bool(torch.isfinite(loss)):
        status |= ST_NONFINITE
    out = {"loss": loss, "chi2": chi2, "chi2_mask": chi2_mask, "model": m, "status": status}
    if return_all:
        out.update({"bx": bx, "by": by, "gx": gx, "gy": gy, "src": s_grid, "f": f,
                    "u": u_img, "transform": tr})
    return out


def obs_from_problem(p) -> dict:
    """Observation dict from a problem produced by the seeded input generator."""
    g = p.geom
    return {"n_img": g.n_img, "pix": float(np.float32(g.pixel_scale)), "ss": g.supersample,
            "image": _t(p.image), "sigma": _t(p.noise_sigma), "psf": _t(p.psf),
            "mask": torch.as_tensor(p.mask.astype(np.int64)), "tau": g.tnfw_tau,
            "n_gauss": getattr(g, "n_gauss", 0), "grid": "uniform" if getattr(g, "uniform", False) else "rtu",
            "ray_weights": None if getattr(p, "ray_weights", None) is None else _t(p.ray_weights),
            "lens_model": "epl" if getattr(g, "epl", False) else "sie"}


def loss_grad(lens, ps, w, obs, n_sub=0, tau=0.0, want_grad=True, return_all=False, cell_shift=0.0,
              picks=None):
    """Loss = chi^2/2 + |w|^2/2 (Gaussian likelihood over all pixels, N(0,1)
    prior on the latent) and its exact gradient with respect to the lens
    parameters, the power-spectrum parameters and the latent field."""
    lens = _t(lens).clone().requires_grad_(want_grad)
    ps = _t(ps).clone().requires_grad_(want_grad)
    w = _t(w).clone().requires_grad_(want_grad)
    out = forward(lens, ps, w, obs, n_sub, tau, return_all=return_all, cell_shift=cell_shift, picks=picks)
    res = {k: v for k, v in out.items()}
    if want_grad:
        gl, gp, gw = torch.autograd.grad(out["loss"], (lens, ps, w), allow_unused=True)
        res["grad_lens"] = gl if gl is not None else torch.zeros_like(lens)
        res["grad_ps"] = gp
        res["grad_latent"] = gw
        for g in (res["grad_lens"], gp, gw):
            if not bool(torch.isfinite(g).all()):
                res["status"] |= ST_NONFINITE
    return res


def loss_grad_problem(p, b: int, want_grad=True, return_all=False, picks=None):
    """loss_grad for sample b of a problem from the seeded input generator."""
    obs = obs_from_problem(p)
    ns = int(p.n_sub[b])
    return loss_grad(p.lens[b].astype(np.float64), p.ps[b].astype(np.float64),
                     p.latent[b].astype(np.float64), obs, ns, p.geom.tnfw_tau,
                     want_grad=want_grad, return_all=return_all, picks=picks)


def position_rounding_bound(lens, ps, w, obs, n_sub=0, tau=0.0):
    """Largest change, in node spacings, of any sub-ray's grid position between
    the exact evaluation and the binary32 rounding model of `forward`."""
    with torch.no_grad():
        a = forward(_t(lens), _t(ps), _t(w), obs, n_sub, tau, return_all=True)
        b = forward(_t(lens), _t(ps), _t(w), obs, n_sub, tau, return_all=True, round32=True)
    n = a["src"].shape[0]
    d = torch.cat([(a["gx"] - b["gx"]).reshape(-1), (a["gy"] - b["gy"]).reshape(-1)]).abs() * n
    d = d[torch.isfinite(d)]
    return float(d.max()) if d.numel() else 0.0


def cell_edge_slack(lens, ps, w, obs, n_sub=0, tau=0.0, delta=None, side=0):
    """How far the lens gradient may move when sub-rays lying within `delta`
    node spacings of a cell edge of the bilinear interpolation (Sec. 2.1) take
    the cell on the other side.

    The interpolant is continuous but its derivative jumps across an edge: a
    position on the edge at column c has d v/d t = s[c] - s[c-1] from the left
    cell and s[c+1] - s[c] from the right one (mixed along the other axis with
    that axis's weights).  An evaluation whose positions carry rounding errors
    of up to `delta` node spacings may therefore give sub-ray r the one-sided
    derivative of either side, which moves d loss/d lens by
        c_r J_r,   c_r = d loss/d v_r * (jump of d v_r/d t_r) * n,
    J_r = d g_r/d lens (through the ray and through the RTU knots).
    Returns sum_r |c_r| |J_r| per lens parameter, the number of sub-ray axes
    within delta of an edge, and delta; delta = None takes twice the
    binary32 rounding model's positional error (position_rounding_bound).
    side = +1 (-1) instead returns the signed first-order change when every
    position within delta below (at or above) an edge takes the cell above
    (below) it: sum of c_r J_r (-c_r J_r) over those sub-rays."""
    if delta is None:
        delta = max(2.0 * position_rounding_bound(lens, ps, w, obs, n_sub, tau), 1e-6)
    lens_t = _t(lens).clone().requires_grad_(False)
    ps_t, w_t = _t(ps), _t(w)
    lens_g = lens_t.clone().requires_grad_(True)
    out = forward(lens_g, ps_t, w_t, obs, n_sub, tau, return_all=True)
    (dldu,) = torch.autograd.grad(out["loss"], [out["u"]])
    N, pix, ss = obs["n_img"], obs["pix"], obs["ss"]
    epl = obs.get("lens_model", "sie") == "epl"
    gx, gy = out["gx"].detach(), out["gy"].detach()
    src = out["src"].detach()
    n = src.shape[0]
    dldv = (dldu.reshape(-1, 1) / (ss * ss)).expand_as(gx)

    def at(i, j):
        ok = (i >= 0) & (i < n) & (j >= 0) & (j < n)
        return torch.where(ok, src.reshape(-1)[torch.where(ok, i * n + j, torch.zeros_like(i))],
                           torch.zeros((), dtype=src.dtype))

    picks = []        # (flat sub-ray index, axis, c_r, below the edge)
    for axis in (0, 1):
        t = (gx if axis == 0 else gy) * n - 0.5
        o = (gy if axis == 0 else gx) * n - 0.5
        c = torch.round(t)
        near = (t - c).abs() < delta
        if not bool(near.any()):
            continue
        ce = c[near].long()
        o0 = torch.floor(o[near])
        fo = o[near] - o0
        o0 = o0.long()

        def val(k, m):   # grid value at (along-axis k, other-axis m)
            return at(m, k) if axis == 0 else at(k, m)

        left = (1 - fo) * (val(ce, o0) - val(ce - 1, o0)) + fo * (val(ce, o0 + 1) - val(ce - 1, o0 + 1))
        right = (1 - fo) * (val(ce + 1, o0) - val(ce, o0)) + fo * (val(ce + 1, o0 + 1) - val(ce, o0 + 1))
        cr = dldv[near] * (right - left) * n
        below = (t - c)[near] < 0
        idx = torch.nonzero(near.reshape(-1)).reshape(-1)
        picks += [(int(i), axis, float(v), bool(lo)) for i, v, lo in zip(idx, cr, below)]
    if not picks:
        return torch.zeros_like(lens_t), 0, delta
    xr, yr = subray_positions(N, pix, ss)
    xr, yr = xr.reshape(-1), yr.reshape(-1)
    mflat = obs["mask"].reshape(-1).bool()
    xc, yc = pixel_centres(N, pix)
    sel = torch.tensor([p[0] for p in picks])
    axes = torch.tensor([p[1] for p in picks])

    rw = obs.get("ray_weights")
    rw = None if rw is None else _t(rw).reshape(-1)[mflat]
    uniform = obs.get("grid", "rtu") == "uniform"

    def g_of(lv):
        bxm, bym = ray_shoot(xc[mflat], yc[mflat], lv, n_sub, tau, epl)
        bx, by = ray_shoot(xr[sel], yr[sel], lv, n_sub, tau, epl)
        if uniform:
            box = uniform_box_of(bxm, bym)
            g1, g2 = (bx - box["lo"][0]) / box["side"], (by - box["lo"][1]) / box["side"]
        else:
            g1, g2 = rtu_transform(bx, by, build_transform(bxm, bym, weights=rw))
        return torch.where(axes == 0, g1, g2)

    J = torch.autograd.functional.jacobian(g_of, lens_t, vectorize=True)     # [picks, n_lens]
    c = torch.tensor([p[2] for p in picks], dtype=DT)
    if side == 0:
        return (c.abs()[:, None] * J.abs()).sum(dim=0), len(picks), delta
    take = torch.tensor([p[3] == (side > 0) for p in picks])
    return (side * (c * take)[:, None] * J).sum(dim=0), int(take.sum()), delta


# ------------------------------------------------------------------ ELBO (Sec. 4)
def elbo_and_grad(mu, rho, eps, obs, n_lens: int, n_sub=0, tau=0.0, log_params=()):
    """Stochastic ELBO of a mean-field Gaussian guide over z = (lens, ps, w)
    with location mu and scale exp(rho), estimated with the given standard-normal
    draws eps[S, dim]:  z_s = mu + exp(rho) eps_s,
        ELBO = -mean_s loss(z_s) - sum_p ln(sigma_p sqrt(2 pi)) - (n^2/2) ln 2 pi
               + sum(rho) + (dim/2)(1 + ln 2 pi),
    i.e. Gaussian likelihood, flat priors on lens and spectrum parameters, a
    unit normal prior on the latent, and the guide entropy.  The lens and
    spectrum parameters listed in log_params (indices into z) have their
    guide over the logarithm:
    z_i = exp(mu_i + exp(rho_i) eps_i), with a flat prior on the logarithm
    (log-uniform on z_i), so the same formula holds.  Returns the ELBO and
    its gradient with respect to mu and rho."""
    mu = _t(mu).clone().requires_grad_(True)
    rho = _t(rho).clone().requires_grad_(True)
    eps = _t(eps)
    S, dim = eps.shape
    nsrc2 = dim - n_lens - 4
    n = int(round(math.sqrt(nsrc2)))
    is_log = torch.zeros(dim, dtype=torch.bool)
    is_log[list(log_params)] = True
    total = torch.zeros((), dtype=DT)
    for s in range(S):
        u = mu + torch.exp(rho) * eps[s]
        z = torch.where(is_log, torch.exp(torch.where(is_log, u, torch.zeros_like(u))), u)
        out = forward(z[:n_lens], z[n_lens:n_lens + 4], z[n_lens + 4:].reshape(n, n),
                      obs, n_sub, tau)
        total = total + out["loss"]
    sig = obs["sigma"]
    const = -torch.log(sig * math.sqrt(2 * math.pi)).sum() - 0.5 * nsrc2 * math.log(2 * math.pi)
    elbo = -total / S + const + rho.sum() + 0.5 * dim * (1.0 + math.log(2 * math.pi))
    gmu, grho = torch.autograd.grad(elbo, (mu, rho))
    return elbo.detach(), gmu, grho


def adam_step(param, grad, m, v, step: int, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) minimising along -grad's
    ascent direction as given (grad is the gradient of the quantity minimised)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return param - lr * mh / (torch.sqrt(vh) + eps), m, v
