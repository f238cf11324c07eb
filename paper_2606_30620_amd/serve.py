"""Serving many RTU-grid lens fits on one GPU.

Requests (a lens system plus the settings of its variational fit) arrive over
time.  `serve_fleet` runs the continuous-batching loop over the library's fleet
(rtu_fleet_*): requests are submitted as they arrive, admitted by the fleet as
its HBM arena and slots free up, advanced together one ELBO + Adam step per
round in shared kernel launches, and retired when done.  `serve_sequential`
is the baseline: one plain fit at a time (rtu_fit_*), in arrival order.

Both return per-request latency (completion - arrival) and the throughput.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, List, Optional

import numpy as np

from . import synth


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float               # seconds after the start of the trace
    problem: synth.Problem
    steps: int
    samples: int = 1
    lr: float = 1e-2
    seed: int = 0

    @property
    def geom(self):
        return self.problem.geom


def log_params(problem: synth.Problem) -> List[int]:
    """Lens parameters fitted in log space: every active subhalo's kappa_s
    and r_s (positive scales; a log-space guide keeps them positive through
    every sample and step)."""
    base = synth.N_LENS_BASE + (1 if problem.geom.epl else 0)
    return [base + synth.N_PER_SUB * j + k for j in range(int(problem.n_sub[0])) for k in (0, 1)]


def guide_init(problem: synth.Problem):
    """Initial guide of a request: location at the request's parameter sample
    (lens, spectrum; the logarithm for the log-space subhalo scales) and the
    latent prior mean; scales 0.01 (lens, spectrum), 0.05 on the logarithm of
    a subhalo scale (5 %) and 1 (latent, the prior's)."""
    g = problem.geom
    lens = problem.lens[0].astype(np.float64).copy()
    rho = np.zeros(lens.size + 4 + g.n_src * g.n_src, np.float32)
    rho[:lens.size + 4] = math.log(0.01)
    for i in log_params(problem):
        lens[i] = math.log(lens[i])
        rho[i] = math.log(0.05)
    mu = np.concatenate([lens, problem.ps[0], np.zeros(g.n_src * g.n_src)]).astype(np.float32)
    return mu, rho


def make_requests(n: int, rate: float, steps: int = 200, samples: int = 1, seed: int = 505,
                  first_id: int = 0, lr: float = 5e-4) -> List[Request]:
    """n requests of the serving mix with Poisson arrivals at `rate` per second
    (rate = inf: all at t = 0).  The step size keeps a fit started at its
    parameter sample inside the parameter domain (subhalo scale radii are a
    few hundredths of an arcsecond)."""
    times = np.zeros(n) if math.isinf(rate) else synth.poisson_arrivals(n, rate, seed)
    return [Request(first_id + i, float(times[i]), synth.serving_request(first_id + i), steps, samples, lr=lr,
                    seed=1000 + first_id + i) for i in range(n)]


def _geometry(lib, g: synth.Geometry):
    return lib.make_geometry(g.n_img, g.supersample, g.n_src, g.psf_size, g.pixel_scale, g.n_sub_max,
                             g.tnfw_tau, flags=(lib.GEOM_UNIFORM if g.uniform else 0) | (lib.GEOM_EPL if g.epl else 0),
                             n_gauss=g.n_gauss)


@dataclasses.dataclass
class ServeResult:
    latency: np.ndarray          # [n] seconds, in request order
    makespan: float              # first arrival -> last completion (s)
    results: dict                # rid -> (mu, rho, elbo trace, status)

    @property
    def fits_per_s(self) -> float:
        return len(self.latency) / self.makespan

    def valid(self) -> Optional[int]:
        """Fits whose samples never left the parameter domain (status bit 8)
        nor gave a non-finite loss or gradient (bit 1), and whose ELBO trace is
        finite; None when the results were not kept.  Bits 2 (smoothed CDF
        not monotone: slopes clamped) and 4 (small mask) are conditions the
        evaluation handles, not failures."""
        if not self.results:
            return None
        return sum(1 for (_, _, tr, st) in self.results.values() if not (st & 9) and np.all(np.isfinite(tr)))

    def status_counts(self) -> dict:
        """Fits with each status bit set in some sample of some step."""
        return {str(b): sum(1 for r in self.results.values() if r[3] & b) for b in (1, 2, 4, 8)}

    def summary(self) -> dict:
        out = {"n": int(len(self.latency)), "fits_per_s": round(self.fits_per_s, 2),
               "p50_ms": round(1e3 * float(np.percentile(self.latency, 50)), 2),
               "p99_ms": round(1e3 * float(np.percentile(self.latency, 99)), 2),
               "makespan_s": round(self.makespan, 3)}
        v = self.valid()
        if v is not None:
            out["valid_fits"] = v
            out["fits_with_status_bit"] = self.status_counts()
        return out


def serve_fleet(requests: List[Request], hbm_budget: int = 8 << 30, max_fits: int = 512, sync_every: int = 4,
                fleet=None, clock: Callable[[], float] = time.perf_counter, keep_results: bool = False,
                sleep: Callable[[float], None] = time.sleep) -> ServeResult:
    """Continuous batching: submit on arrival, run rounds, retire on completion."""
    if fleet is None:
        from . import _lib
        fleet = _lib.Fleet(hbm_budget, max_fits=max_fits, sync_every=sync_every)
    from . import _lib as lib_mod
    reqs = sorted(requests, key=lambda r: r.arrival)
    n = len(reqs)
    arrival = {r.rid: r.arrival for r in reqs}
    done = {}
    results = {}
    ticket_of = {}
    nxt = 0
    t0 = clock()

    def submit_arrived():
        nonlocal nxt
        now = clock() - t0
        while nxt < n and reqs[nxt].arrival <= now:
            r = reqs[nxt]
            mu, rho = guide_init(r.problem)
            p = r.problem
            t = fleet.submit(_geometry(lib_mod, p.geom), p.image, p.noise_sigma, p.psf, p.mask, mu, rho,
                             r.samples, r.steps, int(p.n_sub[0]), r.lr, r.seed, log_params(p))
            ticket_of[t] = r.rid
            nxt += 1

    while len(done) < n:
        submit_arrived()
        st = fleet.stats()
        if st["active"] + st["queued"] == 0:
            if nxt < n:
                sleep(max(0.0, reqs[nxt].arrival - (clock() - t0)))
            continue
        fleet.run(sync_every)
        # requests that arrived meanwhile are prepared on the host while the
        # queued rounds run, and admitted at this sync point
        submit_arrived()
        fleet.sync()
        for t in fleet.poll():
            rid = ticket_of.pop(t)
            done[rid] = clock() - t0
            res = fleet.result(t)
            if keep_results:
                results[rid] = res
    lat = np.array([done[r.rid] - arrival[r.rid] for r in sorted(reqs, key=lambda r: r.rid)])
    first = min(arrival.values())
    return ServeResult(lat, max(done.values()) - first, results)


def serve_sequential(requests: List[Request], clock: Callable[[], float] = time.perf_counter,
                     keep_results: bool = False, sleep: Callable[[float], None] = time.sleep) -> ServeResult:
    """Baseline: each request fitted alone with plain calls, one at a time."""
    from . import _lib
    reqs = sorted(requests, key=lambda r: r.arrival)
    done, results = {}, {}
    t0 = clock()
    for r in reqs:
        wait = r.arrival - (clock() - t0)
        if wait > 0:
            sleep(wait)
        p = r.problem
        plan = _lib.Plan(_geometry(_lib, p.geom), r.samples)
        plan.set_observation(p.image, p.noise_sigma, p.psf, p.mask)
        mu, rho = guide_init(p)
        fit = _lib.Fit(plan, r.samples, mu, rho, lr=r.lr, seed=r.seed, max_steps=r.steps, n_sub=int(p.n_sub[0]),
                       log_params=log_params(p))
        fit.step(r.steps)
        m, rh, tr = fit.read()
        done[r.rid] = clock() - t0
        if keep_results:
            results[r.rid] = (m, rh, tr, fit.status_acc())
        fit.close()
        plan.close()
    lat = np.array([done[r.rid] - r.arrival for r in sorted(reqs, key=lambda r: r.rid)])
    first = min(r.arrival for r in reqs)
    return ServeResult(lat, max(done.values()) - first, results)
