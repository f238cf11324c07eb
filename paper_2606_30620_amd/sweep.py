"""Fit quality against source-grid size, RTU grid versus uniform grid (Sec. 5,
the comparison behind the paper's "about half the pixels per dimension").

A mock is rendered by the library itself: the 200 x 200 geometry of the
headline workload (4 x 4 sub-rays, 21 x 21 PSF, the annulus mask), its true
lens, and a compact source of five knots near the middle of the source plane,
where the caustic concentrates the masked rays (the paper's mocks are
compact galaxies near the caustic).  The knots are spikes in the latent field
of a 256 x 256 uniform grid (Matern n = 1, k0 = 16), so each is the GP
kernel's blob, scaled to a peak brightness of 1; Gaussian noise of arc SNR
13.5 is added.  Neither model grid below contains that source.  Each grid
type and size N_src is then fitted by the library's stochastic variational
fit (Adam on the guide of every parameter; the spectrum's four parameters in
log space, the lens with a guide width of e^-20, i.e. a point estimate,
started at the truth), and the masked reduced chi^2 of the guide mean is
reported with the final ELBO.  Everything that touches
the model runs in the library; this module only sets up inputs and reads
results."""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np


def _problem(base, n_src: int, uniform: bool, lens, ps, latent, image):
    g = dataclasses.replace(base.geom, n_src=n_src, uniform=uniform)
    return dataclasses.replace(base, geom=g, lens=np.asarray(lens, np.float32)[None, :],
                               ps=np.asarray(ps, np.float32)[None, :],
                               latent=np.asarray(latent, np.float32)[None, :, :],
                               n_sub=np.zeros(1, np.int32), image=np.asarray(image, np.float32))


def mock(seed: int = 2606, n_truth: int = 256, k0: float = 16.0, snr: float = 13.5):
    """(problem with the mock image, true lens, true power-spectrum parameters)."""
    import torch

    from . import _lib, api, synth
    base = synth.make_problem("C2", batch=1)
    rng = np.random.default_rng(seed)
    lens = base.lens_truth[:7].astype(np.float32)
    ps = synth.matern_ps_for_k0(k0, 1.0).astype(np.float32)
    c = n_truth // 2
    w = np.zeros((n_truth, n_truth), np.float32)
    for di, dj, a in ((0, 0, 1.0), (-8, 12, 0.7), (12, -10, 0.8), (-18, -18, 0.5), (7, 7, 0.6)):
        w[c + di * n_truth // 256, c + dj * n_truth // 256] = a
    zero = np.zeros_like(base.image)
    res = None
    for _ in range(2):   # the second pass with the knots scaled to a peak brightness of 1
        p = _problem(base, n_truth, True, lens, ps, w, zero)
        plan = api.plan_for_problem(p)
        lt, pt, wt, nt = api.device_inputs(p)
        res = api.evaluate(plan, lt, pt, wt, nt, want_grad=False, want_model=True)
        torch.cuda.synchronize()
        src = plan.debug_fetch(_lib.DBG_SOURCE, 0)
        w = (w / float(src.max())).astype(np.float32)
    model = res.model[0].cpu().numpy().astype(np.float64)
    sigma = float(model[base.mask.astype(bool)].mean()) / snr
    image = model + sigma * rng.standard_normal(model.shape)
    out = dataclasses.replace(base, image=image.astype(np.float32),
                              noise_sigma=np.full_like(base.noise_sigma, sigma))
    return out, lens, ps


def fit_one(problem, lens, ps, n_src: int, uniform: bool, steps: int, samples: int, lr: float, seed: int):
    """Fit one grid; returns the masked reduced chi^2 at the guide mean, the
    last ELBO, the status bits and the wall time."""
    import torch

    from . import _lib, api
    p = _problem(problem, n_src, uniform, lens, ps, np.zeros((n_src, n_src)), problem.image)
    plan = api.plan_for_problem(p, max_batch=samples)
    mu = np.concatenate([lens, ps, np.zeros(n_src * n_src)]).astype(np.float64)
    rho = np.full(mu.size, math.log(0.1))
    rho[:7] = -20.0                       # the lens: a point estimate from the truth
    rho[7:11] = math.log(0.01)
    mu[7:11] = np.log(mu[7:11])          # the spectrum in log space
    fit = _lib.Fit(plan, samples, mu.astype(np.float32), rho.astype(np.float32), lr=lr, seed=seed,
                   max_steps=steps + 1, log_params=[7, 8, 9, 10])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fit.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mu, _, trace = fit.read()
    st = fit.status_acc()
    fit.close()
    ps_fit = np.exp(mu[7:11].astype(np.float64))
    q = _problem(problem, n_src, uniform, mu[:7], ps_fit, mu[11:].reshape(n_src, n_src), problem.image)
    lt, pt, wt, nt = api.device_inputs(q)
    res = api.evaluate(plan, lt, pt, wt, nt, want_grad=False)
    torch.cuda.synchronize()
    return {"chi2_mask": round(float(res.chi2_mask[0]), 4), "elbo_last": round(float(trace[-1]), 2),
            "status_or": int(st), "fit_s": round(wall, 3), "ps_fit": [round(float(v), 5) for v in ps_fit]}


def nsrc_sweep(sizes=(8, 16, 32, 64, 128), steps: int = 3000, samples: int = 4, lr: float = 1e-2,
               seed: int = 7, threshold: float = 2.0) -> dict:
    """The table of both grids over `sizes` (N_src above 64 gets steps x
    N_src / 64 steps), and per grid the smallest N_src whose masked reduced
    chi^2 is within `threshold` of that grid's best."""
    problem, lens, ps = mock()
    rows = {"rtu": {}, "uniform": {}}
    for name, uni in (("rtu", False), ("uniform", True)):
        for n in sizes:
            rows[name][str(n)] = fit_one(problem, lens, ps, n, uni, steps * max(1, n // 64), samples, lr, seed)
    first = {}
    for name, r in rows.items():
        best = min(v["chi2_mask"] for v in r.values())
        first[name] = next(int(n) for n, v in r.items() if v["chi2_mask"] <= threshold * best)
    return {"workload": "200x200 mock: five compact knots on a 256x256 uniform-grid source (Matern n = 1, "
                        "k0 = 16) near the caustic, through the true lens, arc SNR 13.5; fits of N_src x N_src "
                        f"grids, every parameter fitted, {steps} Adam steps, {samples} samples per step",
            "sizes": list(sizes), "table": rows, "chi2_within_factor_of_best": threshold,
            "smallest_n_src_within_factor": first}
