"""Serving fleet on the GPU: each fit's result is the same alone (plain fit
calls) and in a mix of other fits sharing the launches, under admission by an
HBM budget, with arrivals while others run, with a faulty fit in the mix,
and with more admissions at once than the pinned staging pool holds.

Tolerance: ELBO traces within 1e-5 relative, guides within 1e-4 absolute
+ 1e-4 relative (float atomics make any two runs differ at rounding level;
Adam then carries that into the guide)."""
import math

import numpy as np
import pytest

from paper_2606_30620_amd import serve, synth
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

STEPS = 10


def _reqs(ids, samples=2):
    return [serve.Request(i, 0.0, synth.serving_request(i), STEPS, samples, lr=5e-3, seed=900 + i) for i in ids]


def _alone(r):
    from paper_2606_30620_amd import _lib
    p = r.problem
    plan = _lib.Plan(serve._geometry(_lib, p.geom), r.samples)
    plan.set_observation(p.image, p.noise_sigma, p.psf, p.mask)
    mu, rho = serve.guide_init(p)
    fit = _lib.Fit(plan, r.samples, mu, rho, lr=r.lr, seed=r.seed, max_steps=r.steps, n_sub=int(p.n_sub[0]))
    fit.step(r.steps)
    return fit.read()


def _submit(fleet, r):
    from paper_2606_30620_amd import _lib
    p = r.problem
    mu, rho = serve.guide_init(p)
    return fleet.submit(serve._geometry(_lib, p.geom), p.image, p.noise_sigma, p.psf, p.mask, mu, rho,
                        r.samples, r.steps, int(p.n_sub[0]), r.lr, r.seed)


def _same(a, b, what):
    mu_a, rho_a, tr_a = a[:3]
    mu_b, rho_b, tr_b = b[:3]
    assert tr_a.shape == tr_b.shape, what
    assert np.all(np.abs(tr_a - tr_b) <= 1e-5 * np.abs(tr_b) + 1e-6), (what, tr_a, tr_b)
    for x, y in ((mu_a, mu_b), (rho_a, rho_b)):
        assert np.all(np.abs(x - y) <= 1e-4 + 1e-4 * np.abs(y)), (what, np.abs(x - y).max())


def _drain(fleet, tickets, max_rounds=10000):
    out = {}
    rounds = 0
    while len(out) < len(tickets) and rounds < max_rounds:
        fleet.run(4)
        fleet.sync()
        rounds += 4
        for t in fleet.poll():
            out[t] = fleet.result(t)
    assert len(out) == len(tickets), "fleet did not finish"
    return out


def test_alone_equals_mix():
    say("[gpu] fleet: 4 mixed systems in shared launches vs each alone (plain fits)")
    from paper_2606_30620_amd import _lib
    reqs = _reqs([0, 1, 2, 3])
    for r in reqs:
        g = r.geom
        say(f"  req {r.rid}: {g.n_img}^2 ss={g.supersample} n_src={g.n_src} psf={g.psf_size} n_sub={int(r.problem.n_sub[0])}")
    alone = {r.rid: _alone(r) for r in reqs}
    fleet = _lib.Fleet(4 << 30, max_fits=16, sync_every=4)
    tk = {_submit(fleet, r): r.rid for r in reqs}
    got = _drain(fleet, tk)
    for t, res in got.items():
        _same(res, alone[tk[t]], f"request {tk[t]}")
        assert res[3] & 1 == 0


def test_budget_admission_and_midflight_arrivals():
    say("[gpu] fleet: budget for ~2 fits, 5 requests, 2 of them submitted while others run")
    from paper_2606_30620_amd import _lib
    reqs = _reqs([4, 5, 6, 7, 8])
    sizes = []
    for r in reqs:
        p = r.problem
        mu, rho = serve.guide_init(p)
        sizes.append(_lib.Fleet.request_bytes(serve._geometry(_lib, p.geom), p.image, p.noise_sigma, p.psf,
                                              p.mask, mu, rho, r.samples, r.steps, int(p.n_sub[0])))
    budget = int(sorted(sizes)[-1] + sorted(sizes)[-2] + 4096)
    say(f"  request bytes {sizes}, budget {budget}")
    fleet = _lib.Fleet(budget, max_fits=8, sync_every=2)
    tk = {}
    for r in reqs[:3]:
        tk[_submit(fleet, r)] = r.rid
    fleet.run(3)
    st = fleet.stats()
    say(f"  after 3 rounds: {st}")
    assert st["queued"] >= 1 and st["bytes_in_use"] <= budget
    for r in reqs[3:]:
        tk[_submit(fleet, r)] = r.rid
    got = _drain(fleet, tk)
    for t, res in got.items():
        _same(res, _alone([r for r in reqs if r.rid == tk[t]][0]), f"request {tk[t]}")


def test_faulty_fit_does_not_disturb_others():
    say("[gpu] fleet: one fit with a negative Einstein radius in the mix")
    from paper_2606_30620_amd import _lib
    good = _reqs([9, 10])
    bad = _reqs([11])[0]
    fleet = _lib.Fleet(4 << 30, max_fits=8, sync_every=4)
    tk = {_submit(fleet, r): r.rid for r in good}
    p = bad.problem
    mu, rho = serve.guide_init(p)
    mu[0] = -1.0
    tb = fleet.submit(serve._geometry(_lib, p.geom), p.image, p.noise_sigma, p.psf, p.mask, mu, rho,
                      bad.samples, bad.steps, int(p.n_sub[0]), bad.lr, bad.seed)
    got = _drain(fleet, list(tk) + [tb])
    assert got[tb][3] & 8, f"domain status expected, got {got[tb][3]}"
    for t, rid in tk.items():
        _same(got[t], _alone([r for r in good if r.rid == rid][0]), f"request {rid}")


def test_serve_loop_matches_sequential():
    say("[gpu] serve_fleet vs serve_sequential on 6 requests with Poisson arrivals")
    reqs = serve.make_requests(6, rate=200.0, steps=STEPS, samples=1, first_id=20)
    a = serve.serve_fleet(reqs, hbm_budget=2 << 30, max_fits=64, sync_every=4, keep_results=True)
    b = serve.serve_sequential(reqs, keep_results=True)
    say(f"  fleet {a.summary()}  sequential {b.summary()}")
    assert np.all(a.latency > 0) and np.all(b.latency > 0)
    for rid in a.results:
        _same(a.results[rid], b.results[rid], f"request {rid}")


def test_admissions_beyond_the_staging_pool():
    """Ninety fits admitted at one sync point stage more observation data than
    the 64 MiB pinned pool holds (the pool is drained and reused during the
    admissions): each fit's result equals its result in a fleet of its own."""
    from paper_2606_30620_amd import _lib
    ids = [i for i in range(800) if synth.serving_request(i).geom.n_img == 300][:90]
    reqs = [serve.Request(i, 0.0, synth.serving_request(i), 2, 1, lr=5e-3, seed=700 + i) for i in ids]
    staged = sum(r.problem.image.nbytes * 2 + r.problem.mask.nbytes for r in reqs)
    say(f"[gpu] fleet: {len(reqs)} fits of 300 x 300 admitted together ({staged / 2**20:.0f} MiB of image data)")
    assert staged > 64 << 20
    big = _lib.Fleet(6 << 30, max_fits=96, sync_every=4)
    tickets = [_submit(big, r) for r in reqs]
    mix = _drain(big, tickets)
    for r, t in list(zip(reqs, tickets))[::18]:
        own = _lib.Fleet(1 << 30, max_fits=1, sync_every=4)
        alone = _drain(own, [_submit(own, r)])
        _same(mix[t], next(iter(alone.values())), f"request {r.rid}")
