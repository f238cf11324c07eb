"""Pins of the oracle's RTU transform, GP source, interpolation, image and
gradient steps against library routines, closed forms, invariants and brute
force (Sec. 2.1-2.2, eqs. 1-5, App. C)."""
import math

import numpy as np
import pytest
import torch
from scipy import interpolate, signal

from oracle import rtu_oracle as O
from paper_2606_30620_amd import synth

T = lambda a: torch.as_tensor(np.asarray(a), dtype=torch.float64)


# ------------------------------------------------------------ selection (App. C ii)
def test_type7_quantiles_match_numpy_and_hand_example():
    z = T([3.0, 1.0, 4.0, 1.0, 5.0])
    # sorted: 1(i=1) 1(i=3) 3 4 5; u=0.3 -> h=1.2 -> 0.8*1 + 0.2*3 = 1.4
    q, i0, i1 = O.quantiles_type7(z, T([0.3, 0.5, 0.1]))
    assert np.allclose(q.numpy(), [1.4, 3.0, 1.0])
    assert i0.tolist() == [3, 0, 1] and i1.tolist() == [0, 2, 3]   # ties by index
    rng = np.random.default_rng(0)
    zz = rng.standard_normal(1001)
    u = O.chebyshev_nodes()
    q, i0, i1 = O.quantiles_type7(T(zz), u)
    assert np.allclose(q.numpy(), np.quantile(zz, u.numpy(), method="linear"), atol=1e-14)
    # permutation invariance of the values
    perm = rng.permutation(zz.size)
    q2, _, _ = O.quantiles_type7(T(zz[perm]), u)
    assert torch.equal(q, q2)
    # brute force: the selected rays are the order statistics
    srt = np.sort(zz)
    j = np.floor((zz.size - 1) * u.numpy()).astype(int)
    assert np.array_equal(zz[i0.numpy()], srt[j]) and np.array_equal(zz[i1.numpy()], srt[j + 1])


# ------------------------------------------------------------ QF polynomial (iii)
def test_quantiles_with_given_picks():
    """Given order-statistic rays reproduce the sorted selection exactly when
    they are the sorted ones, and give the other order's quantiles when two
    tied rays are swapped (the loss is the same, the selection differs)."""
    rng = np.random.default_rng(4)
    z = T(rng.normal(size=200))
    u = O.chebyshev_nodes()
    q, i0, i1 = O.quantiles_type7(z, u)
    q2, j0, j1 = O.quantiles_type7(z, u, picks=(i0.numpy(), i1.numpy()))
    assert torch.equal(q, q2) and torch.equal(i0, j0) and torch.equal(i1, j1)
    zt = z.clone()
    zt[i1[5]] = zt[i0[5]]                      # a tie at node 5
    q, i0, i1 = O.quantiles_type7(zt, u)
    sw0, sw1 = i0.clone(), i1.clone()
    sw0[5], sw1[5] = i1[5], i0[5]
    q3, _, _ = O.quantiles_type7(zt, u, picks=(sw0.numpy(), sw1.numpy()))
    assert torch.equal(q, q3)
    p = synth.make_problem("C1")
    obs = O.obs_from_problem(p)
    a = O.loss_grad(p.lens[0], p.ps[0], p.latent[0], obs, return_all=True)
    picks = [(a["transform"]["idx"][ax][0].numpy(), a["transform"]["idx"][ax][1].numpy()) for ax in range(2)]
    b = O.loss_grad(p.lens[0], p.ps[0], p.latent[0], obs, picks=picks)
    assert float(a["loss"]) == float(b["loss"]) and torch.equal(a["grad_lens"], b["grad_lens"])


def test_chebyshev_slopes_reproduce_polynomials():
    rng = np.random.default_rng(1)
    u = O.chebyshev_nodes()
    for deg in [1, 5, 21]:
        coef = rng.standard_normal(deg + 1)
        P = np.polynomial.Polynomial(coef)
        q = T(P(u.numpy()))
        dp = O.qf_polynomial(q, u)
        assert np.allclose(dp.numpy(), P.deriv()(u.numpy()), rtol=1e-9, atol=1e-9 * np.abs(coef).sum())


def test_chebyshev_slopes_match_numpy_fit():
    rng = np.random.default_rng(2)
    u = O.chebyshev_nodes()
    q = np.sort(rng.standard_normal(22)) * 2
    fit = np.polynomial.Chebyshev.fit(u.numpy(), q, 21, domain=[0, 1])
    dp = O.qf_polynomial(T(q), u)
    assert np.allclose(dp.numpy(), fit.deriv()(u.numpy()), rtol=1e-8, atol=1e-8)


# ------------------------------------------------------------ spline (iv)
def test_hermite_spline_matches_scipy_and_extrapolates_linearly():
    rng = np.random.default_rng(3)
    X = np.cumsum(rng.uniform(0.1, 0.5, 22))
    u = O.chebyshev_nodes().numpy()
    S = rng.uniform(0.2, 2.0, 22)
    z = rng.uniform(X[0] - 1, X[-1] + 1, 500)
    g = O.cdf_spline(T(z), T(X), T(S), T(u)).numpy()
    ref = interpolate.CubicHermiteSpline(X, u, S)(np.clip(z, X[0], X[-1]))
    inside = (z >= X[0]) & (z <= X[-1])
    assert np.allclose(g[inside], ref[inside], atol=1e-13)
    lo, hi = z < X[0], z > X[-1]
    assert np.allclose(g[lo], u[0] + S[0] * (z[lo] - X[0]), atol=1e-13)
    assert np.allclose(g[hi], u[-1] + S[-1] * (z[hi] - X[-1]), atol=1e-13)
    # values at the knots are the node values
    assert np.allclose(O.cdf_spline(T(X), T(X), T(S), T(u)).numpy(), u, atol=1e-14)


def test_hermite_reproduces_cubics_and_skips_zero_width_intervals():
    cub = lambda z: 0.1 + 0.2 * z + 0.05 * z ** 2 + 0.01 * z ** 3
    dcub = lambda z: 0.2 + 0.1 * z + 0.03 * z ** 2
    X = np.linspace(0.0, 2.0, 22)
    z = np.linspace(0.0, 2.0, 301)
    g = O.cdf_spline(T(z), T(X), T(dcub(X)), T(cub(X))).numpy()
    assert np.allclose(g, cub(z), atol=1e-13)
    # a repeated knot: the interval [X_k, X_k) is never chosen; result stays finite
    X2 = X.copy()
    X2[5] = X2[4]
    g2 = O.cdf_spline(T(X2), T(X2), T(np.ones(22)), T(np.linspace(0, 1, 22))).numpy()
    assert np.isfinite(g2).all()


# ------------------------------------------------------------ whole transform
def _zero_mass_obs(n=48, pix=0.05, ss=1, psf=None, diag=True):
    mask = np.zeros((n, n), np.int64)
    if diag:
        np.fill_diagonal(mask, 1)
    else:
        mask[10:30, 5:40] = 1
    psf = np.zeros((3, 3)) if psf is None else psf
    if psf.sum() == 0:
        psf[1, 1] = 1.0
    return {"n_img": n, "pix": pix, "ss": ss, "image": torch.zeros(n, n, dtype=torch.float64),
            "sigma": torch.ones(n, n, dtype=torch.float64), "psf": T(psf),
            "mask": torch.as_tensor(mask)}


def test_uniform_rays_give_the_uniform_grid():
    """Zero mass and a diagonal mask: the masked projections are distinct and
    equispaced, the quantile function is linear, g is the affine map of the
    masked rays' range onto [0, 1] and the RTU model equals the uniform-grid
    model on that box (Sec. 6.1: the transform tends to the identity)."""
    obs = _zero_mass_obs()
    n, pix = obs["n_img"], obs["pix"]
    lens = T([0.0, 0.1, 0.05, 0.0, 0.0, 0.0, 0.0])      # theta_E = 0: no deflection
    rng = np.random.default_rng(4)
    w = T(rng.standard_normal((16, 16)))
    ps = T(synth.matern_ps_for_k0(4.0, 1.0))
    a = O.forward(lens, ps, w, obs, return_all=True)
    lo = -0.5 * (n - 1) * pix
    b = O.forward(lens, ps, w, obs, uniform_box=(lo, lo, (n - 1) * pix), return_all=True)
    assert torch.allclose(a["gx"], b["gx"], atol=1e-12) and torch.allclose(a["gy"], b["gy"], atol=1e-12)
    assert torch.allclose(a["model"], b["model"], atol=1e-12)
    # end to end: delta PSF and one ray per pixel -> the image is the bilinear
    # sample of the source at the affine-mapped pixel centres
    xc, yc = O.pixel_centres(n, pix)
    ref = O.bilinear(a["src"], (xc - lo) / ((n - 1) * pix), (yc - lo) / ((n - 1) * pix)).reshape(n, n)
    assert torch.allclose(a["model"], ref, atol=1e-12)


def test_transform_invariances_and_knot_values():
    rng = np.random.default_rng(5)
    bxm, bym = T(rng.standard_normal(3000) * 0.7 + 0.2), T(rng.gamma(2.0, 0.4, 3000))
    bx, by = T(rng.uniform(-2, 3, 5000)), T(rng.uniform(-1, 4, 5000))
    tr = O.build_transform(bxm, bym)
    gx, gy = O.rtu_transform(bx, by, tr)
    # affine rescaling of every ray leaves y unchanged (App. C step i)
    a, c = 2.7, T([-0.3, 1.1])
    tr2 = O.build_transform(a * bxm + c[0], a * bym + c[1])
    gx2, gy2 = O.rtu_transform(a * bx + c[0], a * by + c[1], tr2)
    assert torch.allclose(gx, gx2, atol=1e-11) and torch.allclose(gy, gy2, atol=1e-11)
    # the knots map to the node values (Sec. 2.2: the smoothed CDF passes through
    # the eCDF at the nodes)
    u = tr["u"]
    for ax, bm in ((0, bxm), (1, bym)):
        Xb = tr["X"][ax] * tr["s"] + tr["mu"][ax]
        gg = O.rtu_transform(Xb, Xb, tr)[ax]
        assert torch.allclose(gg, u, atol=1e-12)
    # monotone
    zs = T(np.linspace(-5, 5, 2001))
    assert bool((torch.diff(O.rtu_transform(zs, zs, tr)[0]) > 0).all())
    assert tr["status"] == 0


def test_loss_gradient_wrt_standardisation_is_zero():
    """g does not depend on (mu, s): moving them moves knots and rays together."""
    rng = np.random.default_rng(6)
    bxm, bym = T(rng.standard_normal(800)), T(rng.standard_normal(800) * 1.3)
    bx, by = T(rng.uniform(-2, 2, 300)), T(rng.uniform(-2, 2, 300))
    tr = O.build_transform(bxm, bym)
    mu = torch.stack(tr["mu"]).clone().requires_grad_(True)
    s = tr["s"].clone().requires_grad_(True)
    u = tr["u"]
    # rebuild with mu, s as free leaves
    zx, zy = (bxm - mu[0]) / s, (bym - mu[1]) / s
    gsum = 0
    for zm, b, m in ((zx, bx, mu[0]), (zy, by, mu[1])):
        q, _, _ = O.quantiles_type7(zm, u)
        S = 1.0 / O.qf_polynomial(q, u)
        gsum = gsum + (O.cdf_spline((b - m) / s, q, S, u) ** 2).sum()
    gm, gs = torch.autograd.grad(gsum, (mu, s))
    assert gm.abs().max() < 1e-10 and abs(float(gs)) < 1e-10


# ------------------------------------------------------------ GP (eqs. 1-4)
def _dft2(a):
    n = a.shape[0]
    k = np.arange(n)
    W = np.exp(-2j * np.pi * np.outer(k, k) / n)
    return W @ a @ W.T


def test_gp_field_brute_force_dft_and_identities():
    rng = np.random.default_rng(7)
    for n in (4, 8):
        w = rng.standard_normal((n, n))
        sp = rng.uniform(0.5, 2.0, (n, n))
        sp = 0.5 * (sp + np.roll(np.flip(sp), 1, axis=(0, 1)))  # symmetric under k -> -k
        F = _dft2(w)
        Winv = np.conj(np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n))
        ref = (Winv @ (sp * F) @ Winv.T).real / n ** 2
        got = O.gp_field(T(w), T(sp)).numpy()
        assert np.allclose(got, ref, atol=1e-12)
        # P == 1 -> f = w
        assert np.allclose(O.gp_field(T(w), torch.ones(n, n, dtype=torch.float64)).numpy(), w, atol=1e-12)
        # Parseval on the forward transform
        assert np.isclose((np.abs(F) ** 2).sum(), n * n * (w ** 2).sum())


@pytest.mark.parametrize("nm", [0.5, 1.0, 1.5, 2.3])
def test_matern_closed_form(nm):
    """Eq. (4) with 2n/zeta^2 = k0^2 and sigma^2 = A k0^2/(4 pi n) is
    A / (1 + (k/k0)^2)^(n+1); for n = 1 this is the A/(1+(k/k0)^2)^2 spectrum."""
    n, k0, A = 32, 3.0, 2.5
    sig, zeta = math.sqrt(A * k0 * k0 / (4 * math.pi * nm)), math.sqrt(2 * nm) / k0
    sp = O.matern_sqrtP(n, T([sig, nm, zeta, 1.0])).numpy()
    fk = np.fft.fftfreq(n, 1.0 / n)
    k2 = fk[:, None] ** 2 + fk[None, :] ** 2
    assert np.allclose(sp ** 2, A / (1 + k2 / k0 ** 2) ** (nm + 1), rtol=1e-12)


def test_gp_single_mode_amplitude():
    n = 32
    ps = T(synth.matern_ps_for_k0(4.0, 1.0))
    sp = O.matern_sqrtP(n, ps).numpy()
    kx, ky = 3, 5
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    w = np.cos(2 * np.pi * (kx * xx + ky * yy) / n)
    f = O.gp_field(T(w), T(sp)).numpy()
    assert np.allclose(f, sp[ky, kx] * w, atol=1e-12)


def test_gp_sample_variance():
    n, draws = 16, 600
    ps = T(synth.matern_ps_for_k0(4.0, 1.0))
    sp = O.matern_sqrtP(n, ps)
    rng = np.random.default_rng(8)
    fs = np.stack([O.gp_field(T(rng.standard_normal((n, n))), sp).numpy() for _ in range(draws)])
    expect = float((sp ** 2).sum()) / n ** 2
    # per-draw spatial mean of f^2 has mean = expect; compare within 4 sigma
    per = (fs ** 2).mean(axis=(1, 2))
    assert abs(per.mean() - expect) < 4 * per.std() / math.sqrt(draws)


def test_softplus_positivity_transform():
    f = T([-1.0, -0.02, 0.0, 0.003, 0.5])
    for a in (1.0, 1.7):
        s = O.positive_source(f, T(a)).numpy()
        ref = (0.01 * np.log1p(np.exp(f.numpy() / 0.01))) ** a
        assert np.allclose(s, ref, rtol=1e-12, atol=1e-300)


# ------------------------------------------------------------ bilinear (Sec. 2.1)
def test_bilinear_exact_on_linear_fields_and_zero_outside():
    n = 16
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    xs, ys = (j + 0.5) / n, (i + 0.5) / n
    s = 0.3 + 1.7 * xs - 0.9 * ys
    rng = np.random.default_rng(9)
    yx, yy = rng.uniform(0.5 / n, 1 - 0.5 / n, 400), rng.uniform(0.5 / n, 1 - 0.5 / n, 400)
    got = O.bilinear(T(s), T(yx), T(yy)).numpy()
    assert np.allclose(got, 0.3 + 1.7 * yx - 0.9 * yy, atol=1e-13)
    one = O.bilinear(torch.ones(n, n, dtype=torch.float64), T(yx), T(yy)).numpy()
    assert np.allclose(one, 1.0, atol=1e-14)
    far = O.bilinear(torch.ones(n, n, dtype=torch.float64), T([-0.5 / n - 1e-9, 1 + 0.5 / n + 1e-9, 0.5]),
                     T([0.5, 0.5, 1 + 0.5 / n + 1e-6])).numpy()
    assert np.allclose(far, 0.0)
    # half a cell outside the node range: half the edge value
    edge = O.bilinear(torch.ones(n, n, dtype=torch.float64), T([0.0]), T([0.5])).numpy()
    assert np.allclose(edge, 0.5)


# ------------------------------------------------------------ PSF and loss
def test_psf_convolution_brute_force_and_delta():
    rng = np.random.default_rng(10)
    u = rng.standard_normal((20, 23))
    k = rng.standard_normal((5, 5))
    got = O.psf_convolve(T(u), T(k)).numpy()
    ref = signal.convolve2d(u, k, mode="same", boundary="fill")
    assert np.allclose(got, ref, atol=1e-12)
    brute = np.zeros_like(u)
    for a in range(u.shape[0]):
        for b in range(u.shape[1]):
            for p in range(5):
                for q in range(5):
                    ia, jb = a - (p - 2), b - (q - 2)
                    if 0 <= ia < u.shape[0] and 0 <= jb < u.shape[1]:
                        brute[a, b] += k[p, q] * u[ia, jb]
    assert np.allclose(got, brute, atol=1e-12)
    d = np.zeros((5, 5))
    d[2, 2] = 1
    assert np.allclose(O.psf_convolve(T(u), T(d)).numpy(), u)


def test_chi2_zero_when_model_equals_data():
    p = synth.make_problem("C1")
    obs = O.obs_from_problem(p)
    r = O.loss_grad_problem(p, 0, want_grad=False)
    obs["image"] = r["model"].detach()
    r2 = O.loss_grad(p.lens[0], p.ps[0], p.latent[0], obs)
    assert float(r2["chi2"]) < 1e-20
    assert abs(float(r2["loss"]) - 0.5 * float((T(p.latent[0]) ** 2).sum())) < 1e-9
    # the latent gradient is then exactly w (the prior term)
    assert torch.allclose(r2["grad_latent"], T(p.latent[0]), atol=1e-9)


def test_status_bits():
    p = synth.make_problem("C1")
    obs = O.obs_from_problem(p)
    lens = p.lens[0].astype(np.float64).copy()
    lens[0] = -1.0
    assert O.loss_grad(lens, p.ps[0], p.latent[0], obs, want_grad=False)["status"] & O.ST_DOMAIN
    small = dict(obs)
    m = torch.zeros_like(obs["mask"])
    m.view(-1)[:10] = 1
    small["mask"] = m
    st = O.loss_grad(p.lens[0], p.ps[0], p.latent[0], small, want_grad=False)["status"]
    assert st & O.ST_MASK_SMALL


def test_nonmonotone_quantile_function_sets_status_bit_2():
    """Masked rays in two tight clusters make the quantile function a near
    step: the degree-21 interpolant through it overshoots and its slope turns
    negative at some nodes, so the transform clamps those slopes and sets bit 2.
    Unimodal rays give a monotone fit and no bit."""
    rng = np.random.default_rng(5)
    two = np.concatenate([rng.normal(0.0, 0.01, 60), rng.normal(5.0, 0.01, 60)])
    tr = O.build_transform(T(two), T(rng.normal(0.0, 1.0, 120)))
    assert tr["status"] & O.ST_NONMONOTONE
    S = tr["S"][0]
    assert bool((S > 0).all()) and bool(torch.isfinite(S).all())   # clamped, not negative
    dp = O.qf_polynomial(tr["X"][0], tr["u"])
    assert bool((dp <= 1e-6 * (tr["X"][0][-1] - tr["X"][0][0])).any())
    one = O.build_transform(T(rng.normal(0.0, 1.0, 120)), T(rng.normal(0.0, 1.0, 120)))
    assert one["status"] == 0


def test_chebyshev_nodes_match_numpy_first_kind_points():
    """u_k = (1 + x_k)/2 for the Chebyshev points of the first kind x_k
    (numpy's chebpts1), in ascending order."""
    for K in (5, 22):
        ref = 0.5 * (1.0 + np.sort(np.polynomial.chebyshev.chebpts1(K)))
        assert np.allclose(O.chebyshev_nodes(K).numpy(), ref, atol=1e-15, rtol=0)


def test_subray_lattice():
    """Sub-rays: one per pixel at the pixel centre for ss = 1; for ss > 1 a
    regular lattice of spacing pix/ss, centred on the pixel centre (zero mean
    offset), every point inside its pixel."""
    N, pix = 6, 0.07
    xc, yc = O.pixel_centres(N, pix)
    x1, y1 = O.subray_positions(N, pix, 1)
    assert torch.equal(x1[:, 0], xc) and torch.equal(y1[:, 0], yc)
    # pixel (i, j) centre at ((j - (N-1)/2) pix, (i - (N-1)/2) pix), row-major
    assert abs(float(xc[1 * N + 4]) - (4 - 2.5) * pix) < 1e-15
    assert abs(float(yc[1 * N + 4]) - (1 - 2.5) * pix) < 1e-15
    for ss in (2, 3, 4):
        xs, ys = O.subray_positions(N, pix, ss)
        ox, oy = xs - xc[:, None], ys - yc[:, None]
        assert float(ox.mean(1).abs().max()) < 1e-15 and float(oy.mean(1).abs().max()) < 1e-15
        assert float(ox.abs().max()) < 0.5 * pix and float(oy.abs().max()) < 0.5 * pix
        g = ox[0].reshape(ss, ss)                 # sub-ray (a, b) at index a ss + b
        assert torch.allclose(g[:, 1:] - g[:, :-1], torch.full((ss, ss - 1), pix / ss, dtype=torch.float64))
        h = oy[0].reshape(ss, ss)
        assert torch.allclose(h[1:, :] - h[:-1, :], torch.full((ss - 1, ss), pix / ss, dtype=torch.float64))


# ------------------------------------------------------------ gradients
def _fd(fun, x, i, h):
    xp, xm = x.copy(), x.copy()
    xp[i] += h
    xm[i] -= h
    return (fun(xp) - fun(xm)) / (2 * h)


@pytest.mark.parametrize("n_sub", [0, 1])
def test_gradient_matches_central_differences(n_sub):
    """The exact derivative against FP64 central differences.  The loss is only
    piecewise smooth in the lens parameters (the order statistics change
    identity), so lens steps are tiny and a step whose one-sided differences
    disagree (it straddles a kink) is retried smaller."""
    p = synth.make_problem("C1")
    obs = O.obs_from_problem(p)
    lens = p.lens[0].astype(np.float64)
    if n_sub:
        lens = np.concatenate([lens, synth.subhalo_from_mass(3e9, 0.9, 0.5)])
    ps = p.ps[0].astype(np.float64)
    w = p.latent[0].astype(np.float64)
    tau = 10.0 if n_sub else 0.0
    r = O.loss_grad(lens, ps, w, obs, n_sub, tau)
    L = lambda l_, p_, w_: float(O.loss_grad(l_, p_, w_, obs, n_sub, tau, want_grad=False)["loss"])

    for i in range(lens.size):
        ok = False
        for h in (1e-6, 2.5e-7, 6e-8):
            f0 = L(lens, ps, w)
            lp, lm = lens.copy(), lens.copy()
            lp[i] += h
            lm[i] -= h
            fp, fm = L(lp, ps, w), L(lm, ps, w)
            fwd, bwd, cen = (fp - f0) / h, (f0 - fm) / h, (fp - fm) / (2 * h)
            scale = max(abs(cen), 1e-3 * float(r["grad_lens"].abs().max()))
            if abs(fwd - bwd) < 1e-3 * scale:
                assert abs(cen - float(r["grad_lens"][i])) < 2e-4 * scale, (i, cen, float(r["grad_lens"][i]))
                ok = True
                break
        assert ok, f"lens parameter {i}: no kink-free step found"
    for i in range(4):
        cen = _fd(lambda x: L(lens, x, w), ps, i, 1e-6 * max(1.0, abs(ps[i])))
        assert abs(cen - float(r["grad_ps"][i])) < 1e-5 * max(abs(cen), 1.0)
    rng = np.random.default_rng(11)
    for _ in range(6):
        a, b = rng.integers(0, w.shape[0], 2)
        wf = w.reshape(-1)
        cen = _fd(lambda x: L(lens, ps, x.reshape(w.shape)), wf, a * w.shape[0] + b, 1e-5)
        assert abs(cen - float(r["grad_latent"][a, b])) < 1e-5 * max(abs(cen), 1.0)


def test_elbo_with_log_space_parameters():
    """A log-space guide parameter: the loss is taken at z = exp(mu + e^rho eps)
    (the ELBO formula unchanged, flat prior on the logarithm), and the
    gradient in mu agrees with central differences."""
    g = synth.Geometry(48, 0.08, 1, 16, 9, 1.0, n_sub_max=1, tnfw_tau=10.0)
    p = synth.make_problem("X", batch=1, seed=4, geom=g)     # a monotone smoothed CDF (status 0)
    obs = O.obs_from_problem(p)
    n, nl = g.n_src, g.n_lens
    lens = p.lens[0].astype(np.float64).copy()
    logp = [7, 8]
    lens[logp] = np.log(lens[logp])
    mu = np.concatenate([lens, p.ps[0], p.latent[0].reshape(-1)]).astype(np.float64)
    rho = np.full(mu.size, math.log(1e-3))
    eps = np.random.default_rng(13).standard_normal((1, mu.size))
    elbo, gmu, _ = O.elbo_and_grad(mu, rho, eps, obs, nl, 1, g.tnfw_tau, log_params=logp)
    z = mu + np.exp(rho) * eps[0]
    z[logp] = np.exp(z[logp])
    loss = float(O.loss_grad(z[:nl], z[nl:nl + 4], z[nl + 4:].reshape(n, n), obs, 1, g.tnfw_tau,
                             want_grad=False)["loss"])
    sig = p.noise_sigma.astype(np.float64)
    ref = (-loss - np.log(sig * math.sqrt(2 * math.pi)).sum() - 0.5 * n * n * math.log(2 * math.pi)
           + rho.sum() + 0.5 * mu.size * (1 + math.log(2 * math.pi)))
    assert abs(float(elbo) - ref) < 1e-9 * abs(ref)
    assert O.loss_grad(z[:nl], z[nl:nl + 4], z[nl + 4:].reshape(n, n), obs, 1, g.tnfw_tau, want_grad=False)["status"] == 0
    for i in logp:
        cen = _fd(lambda m_: float(O.elbo_and_grad(m_, rho, eps, obs, nl, 1, g.tnfw_tau, log_params=logp)[0]),
                  mu, i, 1e-6)
        assert abs(cen - float(gmu[i])) < 1e-5 * max(1.0, abs(cen)), (i, cen, float(gmu[i]))


def test_elbo_gradient_and_adam():
    p = synth.make_problem("C1")
    obs = O.obs_from_problem(p)
    n = p.geom.n_src
    mu = np.concatenate([p.lens[0], p.ps[0], p.latent[0].reshape(-1)]).astype(np.float64)
    rho = np.full(mu.size, math.log(1e-3))
    rng = np.random.default_rng(12)
    eps = rng.standard_normal((2, mu.size))
    elbo, gmu, grho = O.elbo_and_grad(mu, rho, eps, obs, 7)
    # against the per-sample losses and the guide entropy
    losses = []
    for s in range(2):
        z = mu + np.exp(rho) * eps[s]
        losses.append(float(O.loss_grad(z[:7], z[7:11], z[11:].reshape(n, n), obs, want_grad=False)["loss"]))
    sig = p.noise_sigma.astype(np.float64)
    ref = (-np.mean(losses) - np.log(sig * math.sqrt(2 * math.pi)).sum() - 0.5 * n * n * math.log(2 * math.pi)
           + rho.sum() + 0.5 * mu.size * (1 + math.log(2 * math.pi)))
    assert abs(float(elbo) - ref) < 1e-9 * abs(ref)
    # d ELBO / d rho_i = -mean_s dloss/dz_i * e^rho_i eps_si + 1 ; check on latent entries
    for i in [11, 200, 900]:
        cen = _fd(lambda r_: float(O.elbo_and_grad(mu, r_, eps, obs, 7)[0]), rho, i, 1e-4)
        assert abs(cen - float(grho[i])) < 1e-5 * max(1.0, abs(cen))
        cen = _fd(lambda m_: float(O.elbo_and_grad(m_, rho, eps, obs, 7)[0]), mu, i, 1e-5)
        assert abs(cen - float(gmu[i])) < 1e-5 * max(1.0, abs(cen))
    # Adam against torch.optim.Adam on the same gradient sequence
    x = torch.tensor([0.5, -1.0, 2.0], dtype=torch.float64)
    xt = x.clone().requires_grad_(True)
    opt = torch.optim.Adam([xt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = torch.zeros(3, dtype=torch.float64)
    v = torch.zeros(3, dtype=torch.float64)
    for step in range(1, 6):
        g = torch.tensor([0.3, -2.0, 0.01], dtype=torch.float64) * step
        x, m, v = O.adam_step(x, g, m, v, step)
        opt.zero_grad()
        xt.grad = g.clone()
        opt.step()
    assert torch.allclose(x, xt.detach(), atol=1e-15)


def test_cell_edge_slack_predicts_one_sided_derivative_flips():
    """Pin of the oracle's cell-edge bound: moving every sub-ray position that
    lies within delta below (above) a bilinear cell edge into the cell above
    (below) changes the lens gradient, computed by autograd through the
    shifted interpolation, by the signed first-order sum the bound is built
    from; and the absolute bound dominates both changes."""
    p = synth.make_problem("C1")
    obs = O.obs_from_problem(p)
    args = (p.lens[0].astype(np.float64), p.ps[0].astype(np.float64), p.latent[0].astype(np.float64), obs,
            int(p.n_sub[0]), p.geom.tnfw_tau)
    delta = 1e-3
    g0 = O.loss_grad(*args)["grad_lens"].detach().numpy()
    bound, n, _ = O.cell_edge_slack(*args, delta=delta)
    assert n > 0
    for side in (1, -1):
        pred, m, _ = O.cell_edge_slack(*args, delta=delta, side=side)
        got = O.loss_grad(*args, cell_shift=side * delta)["grad_lens"].detach().numpy() - g0
        assert m > 0
        np.testing.assert_allclose(pred.numpy(), got, rtol=0, atol=5e-3 * np.abs(got).max())
        assert np.all(np.abs(got) <= bound.numpy() * 1.01)
    # the binary32 rounding model moves positions by far less than a cell
    r = O.position_rounding_bound(*args)
    assert 0 < r < 1e-3
