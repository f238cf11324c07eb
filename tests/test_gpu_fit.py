"""The ELBO + Adam fit step on the GPU against the oracle's ELBO and its
gradient (Sec. 4), with the standard-normal draws passed in to both sides;
checkpoint/resume; the on-device Philox normal draws."""
import math

import numpy as np
import pytest
import torch

from oracle import rtu_oracle as O
from paper_2606_30620_amd import synth
from tests.gpu_helpers import relinf, say
from tests.test_gpu_parity import c1_mock

pytestmark = pytest.mark.gpu


def _guide(p, rho_val=math.log(1e-3)):
    mu = np.concatenate([p.lens[0], p.ps[0], p.latent[0].reshape(-1)]).astype(np.float64)
    return mu, np.full(mu.size, rho_val)


def test_elbo_step_matches_oracle():
    say("[gpu] fit: one ELBO+Adam step, C1, S=2, eps given")
    _elbo_step_check(c1_mock(), {"lens": slice(0, 7), "ps": slice(7, 11), "latent": slice(11, None)})


def test_elbo_step_with_lens_light_matches_oracle():
    say("[gpu] fit: one ELBO+Adam step with 3 lens-light Gaussians, 48x48 ss=2 n_src=16, S=2, eps given")
    g = synth.Geometry(48, 0.08, 2, 16, 15, 1.0, n_gauss=3)
    p = synth.make_problem("X", batch=1, seed=31, geom=g)
    _elbo_step_check(p, {"lens": slice(0, 7), "light": slice(7, 25), "ps": slice(25, 29),
                         "latent": slice(29, None)})


def test_elbo_step_with_log_space_subhalo_scales_matches_oracle():
    """Subhalo kappa_s and r_s fitted in log space (z = exp(u), flat prior on u):
    the sampled scales are exp of the guide's draws, the gradient is chained
    through z, and one step agrees with the oracle's ELBO for that guide."""
    say("[gpu] fit: one ELBO+Adam step, 2 subhaloes with log-space kappa_s and r_s, 64x64 ss=2 n_src=16, S=2")
    g = synth.Geometry(64, 0.06, 2, 16, 15, 1.0, n_sub_max=2, tnfw_tau=10.0)
    p = synth.make_problem("X", batch=1, seed=33, geom=g)
    _elbo_step_check(p, {"lens": slice(0, 7), "subhaloes": slice(7, 15), "ps": slice(15, 19),
                         "latent": slice(19, None)}, log_params=[7, 8, 11, 12], n_sub=2)


def test_elbo_step_with_log_space_spectrum_matches_oracle():
    """The power spectrum's sigma and zeta in log space as well."""
    say("[gpu] fit: one ELBO+Adam step, log-space spectrum sigma and zeta, 48x48 ss=2 n_src=16, S=2")
    g = synth.Geometry(48, 0.08, 2, 16, 15, 1.0)
    p = synth.make_problem("X", batch=1, seed=35, geom=g)
    _elbo_step_check(p, {"lens": slice(0, 7), "ps": slice(7, 11), "latent": slice(11, None)},
                     log_params=[7, 9])


@pytest.mark.parametrize("S", [5, 19])
def test_elbo_step_sample_counts(S):
    """Sample counts that leave some of the Adam update's sample groups
    short or idle (5: eight groups; 19: sixteen groups, three of them with
    two samples)."""
    say(f"[gpu] fit: one ELBO+Adam step, C1, S={S}, eps given")
    _elbo_step_check(c1_mock(), {"lens": slice(0, 7), "ps": slice(7, 11), "latent": slice(11, None)}, S=S)


def _elbo_step_check(p, groups, log_params=(), n_sub=0, S=2):
    from paper_2606_30620_amd import _lib, api
    plan = api.plan_for_problem(p, max_batch=S)
    mu, rho = _guide(p)
    for i in log_params:
        mu[i] = math.log(mu[i])
        rho[i] = math.log(0.05)
    mu32, rho32 = mu.astype(np.float32), rho.astype(np.float32)
    rng = np.random.default_rng(21)
    eps = rng.standard_normal((S, mu.size)).astype(np.float32)
    fit = _lib.Fit(plan, S, mu32, rho32, lr=1e-2, seed=1, max_steps=4, n_sub=n_sub, log_params=log_params)
    fit.step(1, eps=torch.from_numpy(eps).cuda())
    state, steps = fit.get_state()
    _, _, trace = fit.read()
    assert steps == 1 and trace.size == 1
    obs = O.obs_from_problem(p)
    elbo, gmu, grho = O.elbo_and_grad(mu32.astype(np.float64), rho32.astype(np.float64),
                                      eps.astype(np.float64), obs, p.geom.n_lens, n_sub, p.geom.tnfw_tau,
                                      log_params=log_params)
    if log_params:
        z = fit.samples()
        u = mu32[None, :].astype(np.float64) + np.exp(rho32.astype(np.float64))[None, :] * eps
        assert np.allclose(z[:, log_params], np.exp(u[:, log_params]), rtol=1e-5)
    # after one step from zero moments, m = (1 - 0.9) * d(-ELBO)/d(param)
    m_mu, m_rho = state[2] / 0.1, state[4] / 0.1
    ref_mu, ref_rho = -gmu.numpy(), -grho.numpy()
    for name, sl in groups.items():
        e1 = relinf(m_mu[sl], ref_mu[sl])
        e2 = relinf(m_rho[sl] + 1.0, ref_rho[sl] + 1.0)     # remove the entropy term's -1
        say(f"  grad mu[{name}] {e1:.2e}   grad rho[{name}] {e2:.2e}")
        assert e1 <= 1e-3 and e2 <= 1e-3, name
    el_ref = float(elbo)
    say(f"  elbo gpu {trace[0]:.6f} oracle {el_ref:.6f}")
    assert abs(trace[0] - el_ref) <= 1e-4 * max(abs(el_ref), 1.0)
    # Adam arithmetic on the GPU's own moments
    c1, c2 = 1 / (1 - 0.9), 1 / (1 - 0.999)
    exp_mu = mu32 - 1e-2 * (state[2] * c1) / (np.sqrt(state[3] * c2) + 1e-8)
    assert np.allclose(state[0], exp_mu, atol=1e-6)


def test_checkpoint_resume_is_bitwise():
    say("[gpu] fit: 3 steps == 2 steps + save + restore into a new fit + 1 step (Philox draws)")
    from paper_2606_30620_amd import _lib, api
    p = c1_mock()
    plan = api.plan_for_problem(p, max_batch=4)
    mu, rho = _guide(p, math.log(1e-2))
    a = _lib.Fit(plan, 4, mu, rho, lr=5e-3, seed=77, max_steps=8)
    a.step(3)
    sa, na = a.get_state()
    b = _lib.Fit(plan, 4, mu, rho, lr=5e-3, seed=77, max_steps=8)
    b.step(2)
    ckpt, nb = b.get_state()
    c = _lib.Fit(plan, 4, mu * 0, rho * 0, lr=5e-3, seed=77, max_steps=8)
    c.set_state(ckpt, nb)
    c.step(1)
    sc, nc = c.get_state()
    assert na == nc == 3
    # mu, rho and the moments agree to float rounding (float atomics in the
    # gradient sum make runs differ in the last bits)
    for k in range(6):
        assert relinf(sc[k], sa[k]) < 1e-4, k


def test_fit_decreases_negative_elbo():
    say("[gpu] fit: 60 steps of C1 from a perturbed start raise the ELBO")
    from paper_2606_30620_amd import _lib, api
    p = c1_mock()
    plan = api.plan_for_problem(p, max_batch=4)
    mu, rho = _guide(p, math.log(1e-3))
    fit = _lib.Fit(plan, 4, mu, rho, lr=2e-3, seed=5, max_steps=100)
    fit.step(60)
    _, _, tr = fit.read()
    say(f"  ELBO first {tr[0]:.1f} last {tr[-1]:.1f}")
    assert np.all(np.isfinite(tr))
    assert tr[-5:].mean() > tr[:5].mean()


def test_philox_normals_statistics():
    say("[gpu] Philox draws: mean 0, variance 1, no correlation between samples or steps")
    from paper_2606_30620_amd import _lib, api
    p = c1_mock()
    plan = api.plan_for_problem(p, max_batch=8)
    mu = np.concatenate([p.lens[0], p.ps[0], np.zeros(32 * 32)]).astype(np.float32)
    rho = np.full(mu.size, -30.0, np.float32)
    rho[11:] = 0.0                    # latent part: z = eps exactly
    fit = _lib.Fit(plan, 8, mu, rho, lr=0.0, seed=123, max_steps=2)
    fit.step(1)
    z1 = fit.samples()[:, 11:].astype(np.float64)
    fit.step(1)
    z2 = fit.samples()[:, 11:].astype(np.float64)
    for z in (z1, z2):
        n = z.size
        assert abs(z.mean()) < 4 / math.sqrt(n)
        assert abs(z.var() - 1.0) < 4 * math.sqrt(2.0 / n)
    c = np.corrcoef(np.concatenate([z1, z2]))
    off = c[~np.eye(16, dtype=bool)]
    assert np.abs(off).max() < 5 / math.sqrt(z1.shape[1])
    # a different seed gives different draws
    f2 = _lib.Fit(plan, 8, mu, rho, lr=0.0, seed=124, max_steps=1)
    f2.step(1)
    assert not np.array_equal(f2.samples()[:, 11:], z1.astype(np.float32))
