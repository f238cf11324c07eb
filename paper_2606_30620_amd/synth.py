"""Seeded synthetic inputs for the RTU-grid lens likelihood.

This module holds no lensing or source-model arithmetic.  It only draws
parameters, noise and simple image-plane shapes from a seeded numpy
generator, so that the GPU library and the FP64 oracle can be fed
identical inputs.  Every floating-point array is rounded to float32 here,
so both sides see the same values.

Workloads (sizes follow the paper's mock set-up, Sec. 3.1: 200x200 pixels of
0.031 arcsec with a PSF of FWHM twice the pixel width; arc masks as in
Sec. 3.1, replaced here by an annulus around the true lens):

* ``C1``  64x64 at 0.05"/px, 1 ray per pixel, 32x32 source, 15x15 PSF, 1 sample.
* ``C2``  200x200 at 0.031"/px, 4x4 sub-rays, 64x64 source, 21x21 PSF,
          32 latent samples; lens drawn uniformly.
* ``C3``  400x400 at 0.0155"/px, 3x3 sub-rays, 128x128 source, 31x31 PSF,
          1..10 truncated-NFW subhaloes.
* ``C4``  512x512 at 0.01211"/px, 4x4 sub-rays, 256x256 source,
          Matern-3/2-like spectrum, 64 samples.
* ``C5``  serving mix: image, sub-ray, source and subhalo counts drawn per
          request.

The observed image of C2..C5 is an arc-like ring (an elliptical Gaussian
ring with azimuthal modulation and two compact knots) plus Gaussian noise
whose sigma gives an average arc SNR of 13.5 (the paper's mocks have
SNR 12-15 over the arcs).  It is synthetic data of the right size and
structure, not a lensed mock.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

#: number of lens parameters before the subhaloes:
#: theta_E, e1, e2, x0, y0, gamma1, gamma2
N_LENS_BASE = 7
#: parameters per subhalo: kappa_s, r_s, x_s, y_s
N_PER_SUB = 4
#: power-spectrum parameters: sigma_src, n_src, zeta_src, alpha_src
N_PS = 4
#: parameters per lens-light Gaussian: A, sigma, e1, e2, x_c, y_c (after the
#: subhalo slots in the lens vector)
N_PER_GAUSS = 6


@dataclasses.dataclass(frozen=True)
class Geometry:
    n_img: int
    pixel_scale: float      # arcsec per image pixel
    supersample: int        # sub-rays per pixel along each axis
    n_src: int              # source grid pixels per side (power of two)
    psf_size: int           # odd PSF kernel width in pixels
    psf_sigma_px: float     # Gaussian PSF sigma in image pixels
    n_sub_max: int = 0
    tnfw_tau: float = 0.0   # truncation radius in units of r_s; 0 = none
    n_gauss: int = 0        # lens-light Gaussians; 0 = no lens light
    uniform: bool = False   # source grid on the masked rays' square box instead of the RTU grid
    epl: bool = False       # main deflector: elliptical power law, its slope as lens parameter 7

    @property
    def n_lens(self) -> int:
        return N_LENS_BASE + (1 if self.epl else 0) + N_PER_SUB * self.n_sub_max + N_PER_GAUSS * self.n_gauss


def e_from_q_phi(q: float, phi: float):
    """(q, phi) -> (e1, e2) with e = (1-q)/(1+q), (e1, e2) = e (cos 2phi, sin 2phi)."""
    e = (1.0 - q) / (1.0 + q)
    return e * math.cos(2.0 * phi), e * math.sin(2.0 * phi)


def matern_ps_for_k0(k0: float, n: float, amplitude: float = 1.0, alpha: float = 1.0):
    """Power-spectrum parameters whose Matern spectrum equals
    amplitude / (1 + (k/k0)^2)^(n+1).

    This is parameter bookkeeping only: 2n/zeta^2 = k0^2 and
    sigma^2 4 pi n / k0^2 = amplitude.
    """
    zeta = math.sqrt(2.0 * n) / k0
    sigma = math.sqrt(amplitude * k0 * k0 / (4.0 * math.pi * n))
    return np.array([sigma, n, zeta, alpha], dtype=np.float64)


def pixel_centres(n_img: int, pix: float):
    """Pixel-centre coordinates (x, y) in arcsec, row i <-> y, column j <-> x,
    centred on the image centre."""
    c = (np.arange(n_img, dtype=np.float64) - 0.5 * (n_img - 1)) * pix
    y, x = np.meshgrid(c, c, indexing="ij")
    return x, y


def annulus_mask(n_img: int, pix: float, centre, theta_e: float,
                 r_in: float = 0.5, r_out: float = 1.5) -> np.ndarray:
    """uint8 mask of pixels with r_in*theta_E <= |theta - centre| <= r_out*theta_E."""
    x, y = pixel_centres(n_img, pix)
    r = np.hypot(x - centre[0], y - centre[1])
    return ((r >= r_in * theta_e) & (r <= r_out * theta_e)).astype(np.uint8)


def gaussian_psf(size: int, sigma_px: float) -> np.ndarray:
    h = np.arange(size, dtype=np.float64) - (size - 1) / 2
    g = np.exp(-0.5 * (h / sigma_px) ** 2)
    k = np.outer(g, g)
    return k / k.sum()


def arc_image(n_img: int, pix: float, lens_truth: np.ndarray, rng) -> np.ndarray:
    """A noiseless arc-like ring around the lens (no lensing computation)."""
    x, y = pixel_centres(n_img, pix)
    the, e1, e2, x0, y0 = lens_truth[:5]
    e = math.hypot(e1, e2)
    q = (1 - e) / (1 + e)
    phi = 0.5 * math.atan2(e2, e1)
    dx, dy = x - x0, y - y0
    xp = math.cos(phi) * dx + math.sin(phi) * dy
    yp = -math.sin(phi) * dx + math.cos(phi) * dy
    rho = np.sqrt(q * xp * xp + yp * yp / q)
    ang = np.arctan2(yp, xp)
    width = 0.08 * the
    a0 = rng.uniform(0, 2 * np.pi)
    ring = np.exp(-0.5 * ((rho - the) / width) ** 2) * (1.0 + 0.6 * np.cos(2 * (ang - a0)))
    for _ in range(2):
        ak = rng.uniform(0, 2 * np.pi)
        cx, cy = x0 + the * math.cos(ak), y0 + the * math.sin(ak)
        ring += 1.5 * np.exp(-0.5 * ((x - cx) ** 2 + (y - cy) ** 2) / (0.05 * the) ** 2)
    return ring


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


@dataclasses.dataclass
class Problem:
    """One lens system with B parameter samples."""
    geom: Geometry
    image: np.ndarray        # float32 [N, N]
    noise_sigma: np.ndarray  # float32 [N, N]
    psf: np.ndarray          # float32 [K, K]
    mask: np.ndarray         # uint8   [N, N]
    lens: np.ndarray         # float32 [B, n_lens]
    n_sub: np.ndarray        # int32   [B]
    ps: np.ndarray           # float32 [B, 4]
    latent: np.ndarray       # float32 [B, n_src, n_src]
    lens_truth: np.ndarray   # float64 [n_lens]
    noise: Optional[np.ndarray] = None  # float32 [N, N] unit-free noise draw (C1)
    ray_weights: Optional[np.ndarray] = None  # float32 [N, N] weights of the masked rays (weighted RTU grid)

    @property
    def batch(self) -> int:
        return self.lens.shape[0]


def _perturb_lens(rng, truth, B, n_sub_max):
    """Per-sample lens parameters around the truth (the spread of a Gaussian
    guide at a random, non-optimal point)."""
    scale = np.array([0.02, 0.02, 0.02, 0.01, 0.01, 0.01, 0.01]
                     + [0.0, 0.0, 0.01, 0.01] * n_sub_max)
    lens = truth[None, :] + rng.standard_normal((B, truth.size)) * scale[None, :]
    for j in range(n_sub_max):  # multiplicative spread for positive kappa_s, r_s
        b = N_LENS_BASE + N_PER_SUB * j
        lens[:, b:b + 2] = truth[None, b:b + 2] * np.exp(0.05 * rng.standard_normal((B, 2)))
    return lens


def _perturb_ps(rng, ps_truth, B):
    return ps_truth[None, :] * np.exp(0.05 * rng.standard_normal((B, N_PS)))


def sie_truth(rng, centre_jitter=0.05):
    the = rng.uniform(0.6, 1.6)
    q = rng.uniform(0.5, 0.95)
    phi = rng.uniform(0.0, math.pi)
    e1, e2 = e_from_q_phi(q, phi)
    r = 0.08 * math.sqrt(rng.uniform())
    a = rng.uniform(0, 2 * math.pi)
    x0, y0 = rng.uniform(-centre_jitter, centre_jitter, 2)
    return np.array([the, e1, e2, x0, y0, r * math.cos(a), r * math.sin(a)])


NFW_H1 = 1.0 + math.log(0.5)  # projected-mass function of the NFW profile at x = 1


def subhalo_from_mass(mass_msun: float, xs: float, ys: float):
    """Subhalo (kappa_s, r_s, x_s, y_s) for a mass given as an equivalent
    Einstein radius: theta_E,sub = 1" sqrt(M / 1e11 Msun), r_s = theta_E,sub and
    kappa_s = 1 / (4 h(1)) so the mean convergence inside theta_E,sub is one."""
    te = math.sqrt(mass_msun / 1e11)
    return [1.0 / (4.0 * NFW_H1), te, xs, ys]


def _subhaloes(rng, n_sub, n_sub_max):
    out = []
    for j in range(n_sub_max):
        m = 10 ** rng.uniform(8, 10)
        r = 1.5 * math.sqrt(rng.uniform())
        a = rng.uniform(0, 2 * math.pi)
        sh = subhalo_from_mass(m, r * math.cos(a), r * math.sin(a))
        if j >= n_sub:
            sh = [0.0, 1.0, 0.0, 0.0]   # padding slot (ignored: beyond n_sub)
        out += sh
    return np.array(out, dtype=np.float64)


def _light_truth(rng, n_gauss, centre):
    """Lens-light Gaussians: widths log-uniform in [0.1, 1.0] arcsec and sorted
    (the paper's prior range), amplitudes, mildly elliptical, centred near the
    lens."""
    sig = np.sort(10 ** rng.uniform(-1.0, 0.0, n_gauss))
    out = []
    for n in range(n_gauss):
        e1, e2 = e_from_q_phi(rng.uniform(0.7, 0.95), rng.uniform(0.0, math.pi))
        cx, cy = np.asarray(centre) + rng.uniform(-0.02, 0.02, 2)
        out += [rng.uniform(0.5, 2.0), sig[n], e1, e2, cx, cy]
    return np.array(out, dtype=np.float64)


def _light_image(n_img, pix, light):
    """Noiseless image of the lens-light Gaussians at the pixel centres (data
    only: an elliptical Gaussian blob per component)."""
    x, y = pixel_centres(n_img, pix)
    img = np.zeros_like(x)
    for n in range(light.size // N_PER_GAUSS):
        A, sig, e1, e2, cx, cy = light[N_PER_GAUSS * n:N_PER_GAUSS * (n + 1)]
        e = math.hypot(e1, e2)
        q = (1 - e) / (1 + e)
        phi = 0.5 * math.atan2(e2, e1)
        dx, dy = x - cx, y - cy
        xp = math.cos(phi) * dx + math.sin(phi) * dy
        yp = -math.sin(phi) * dx + math.cos(phi) * dy
        img += A / (2 * math.pi) * np.exp(-0.5 * (q * xp * xp + yp * yp / q) / sig ** 2)
    return img


CONFIGS = {
    "C1": Geometry(64, 0.05, 1, 32, 15, 1.6),
    "C2": Geometry(200, 0.031, 4, 64, 21, 2.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))),
    "C3": Geometry(400, 0.0155, 3, 128, 31, 2.0 / (2.0 * math.sqrt(2.0 * math.log(2.0))),
                   n_sub_max=10, tnfw_tau=10.0),
    "C4": Geometry(512, 0.01211, 4, 256, 21, 2.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))),
}
SEEDS = {"C1": 101, "C2": 202, "C3": 303, "C4": 404, "C5": 505}
DEFAULT_BATCH = {"C1": 1, "C2": 32, "C3": 32, "C4": 64}


def make_problem(name: str, batch: Optional[int] = None, seed: Optional[int] = None,
                 geom: Optional[Geometry] = None) -> Problem:
    """Build the seeded inputs of a named workload (see module docstring)."""
    geom = geom or CONFIGS[name]
    B = DEFAULT_BATCH.get(name, 1) if batch is None else batch
    rng = np.random.default_rng(SEEDS.get(name, 0) if seed is None else seed)
    N, pix = geom.n_img, geom.pixel_scale
    psf = gaussian_psf(geom.psf_size, geom.psf_sigma_px)
    if name == "C1":
        e1, e2 = e_from_q_phi(0.8, math.radians(30.0))
        truth = np.array([1.0, e1, e2, 0.0, 0.0, 0.03, -0.01])
        ps = matern_ps_for_k0(4.0, 1.0)[None, :].repeat(B, 0)
        lens = truth[None, :].repeat(B, 0)
        mask = annulus_mask(N, pix, (0.0, 0.0), 1.0)
        latent = rng.standard_normal((B, geom.n_src, geom.n_src))
        noise = rng.standard_normal((N, N)) * 0.01
        # C1's observed image is the model plus this noise; the caller renders
        # the model.  Until then the image slot holds the noise alone.
        image = noise.copy()
        sigma = np.full((N, N), 0.01)
        return Problem(geom, _f32(image), _f32(sigma), _f32(psf), mask,
                       _f32(lens), np.zeros(B, np.int32), _f32(ps), _f32(latent),
                       truth, noise=_f32(noise))
    truth = sie_truth(rng)
    n_sub = np.zeros(B, np.int32)
    if geom.n_sub_max:
        ns = int(rng.integers(1, geom.n_sub_max + 1))
        truth = np.concatenate([truth, _subhaloes(rng, ns, geom.n_sub_max)])
        n_sub[:] = ns
    if name == "C4":
        ps_truth = matern_ps_for_k0(4.0, 1.5)
    else:
        ps_truth = matern_ps_for_k0(4.0, 1.0)
    lens = _perturb_lens(rng, truth, B, geom.n_sub_max)
    ps = _perturb_ps(rng, ps_truth, B)
    latent = rng.standard_normal((B, geom.n_src, geom.n_src))
    mask = annulus_mask(N, pix, truth[3:5], truth[0])
    clean = arc_image(N, pix, truth, rng)
    if geom.n_gauss:
        light = _light_truth(rng, geom.n_gauss, truth[3:5])
        truth = np.concatenate([truth, light])
        spread = np.tile([0.02, 0.02, 0.01, 0.01, 0.005, 0.005], geom.n_gauss)
        lens = np.concatenate([lens, light[None, :] * np.ones((B, 1))
                               + rng.standard_normal((B, light.size)) * spread[None, :]
                               * np.tile([light[0], light[1], 1, 1, 1, 1], geom.n_gauss)[None, :]], axis=1)
        clean = clean + _light_image(N, pix, light)
    sig = float(clean[mask.astype(bool)].mean()) / 13.5
    image = clean + sig * rng.standard_normal((N, N))
    sigma = np.full((N, N), sig)
    return Problem(geom, _f32(image), _f32(sigma), _f32(psf), mask,
                   _f32(lens), n_sub, _f32(ps), _f32(latent), truth)


def with_epl(problem: Problem, slope_mean: float = 2.1, slope_spread: float = 0.05, seed: int = 77) -> Problem:
    """The same system with the EPL deflector: a slope per sample (drawn
    around slope_mean) inserted as lens parameter 7, the subhaloes and lens
    light moved up by one."""
    rng = np.random.default_rng(seed)
    B = problem.batch
    g = rng.normal(slope_mean, slope_spread, B)
    lens = np.concatenate([problem.lens[:, :N_LENS_BASE], g[:, None], problem.lens[:, N_LENS_BASE:]], axis=1)
    truth = np.concatenate([problem.lens_truth[:N_LENS_BASE], [slope_mean], problem.lens_truth[N_LENS_BASE:]])
    return dataclasses.replace(problem, geom=dataclasses.replace(problem.geom, epl=True), lens=_f32(lens),
                               lens_truth=truth)


# ---------------------------------------------------------------- serving mix
C5_IMG = (64, 100, 150, 200, 300)
C5_SS = (2, 3, 4)
C5_SRC = (32, 64, 128)


def serving_request(req_id: int, field_arcsec: float = 6.2, n_sub_cap: int = 3) -> Problem:
    """One request of the serving mix (seed 1000 + id): image size, sub-rays,
    source size and 0..3 subhaloes drawn per request, one parameter sample."""
    rng = np.random.default_rng(1000 + req_id)
    N = int(rng.choice(C5_IMG))
    ss = int(rng.choice(C5_SS))
    ns = int(rng.choice(C5_SRC))
    nsub = int(rng.integers(0, n_sub_cap + 1))
    pix = field_arcsec / N
    geom = Geometry(N, pix, ss, ns, 21 if N >= 150 else 15,
                    2.0 / (2.0 * math.sqrt(2.0 * math.log(2.0))),
                    n_sub_max=nsub, tnfw_tau=10.0 if nsub else 0.0)
    return make_problem("C5", batch=1, seed=int(rng.integers(1 << 31)), geom=geom)


def poisson_arrivals(n: int, rate_per_s: float, seed: int = 505) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))
