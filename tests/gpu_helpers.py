"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compare it with the FP64 oracle sample by sample."""
from __future__ import annotations

import sys

import numpy as np
import torch

from oracle import rtu_oracle as O

TOL_IMG = 1e-4    # images and loss: |diff|_inf / |ref|_inf
TOL_GRAD = 1e-3   # gradients: per group, |diff|_inf / |ref group|_inf
TIE_REL = 2e-5    # two order statistics closer than this (relative to the
                  # masked rays' range) may legitimately swap between FP32 and FP64
SLACK_MAX = 5.0   # the cell-edge allowance may add at most this many TOL_GRAD


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def relinf(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = np.abs(a - b).max()
    s = np.abs(b).max()
    return d / s if s > 0 else d


def selection_agrees(gpu_sel, tr, z_axes):
    """True if the GPU picked the same rays as the oracle; raises if a differing
    pick is not a near-tie (not a valid alternative order statistic)."""
    same = True
    for ax in range(2):
        i0, i1 = tr["idx"][ax]
        ref = np.stack([i0.numpy(), i1.numpy()], axis=1).reshape(-1)
        got = gpu_sel[ax]
        z = z_axes[ax]
        rng = float(z.max() - z.min())
        for r in range(ref.size):
            if got[r] != ref[r]:
                same = False
                gap = abs(float(z[got[r]] - z[ref[r]]))
                assert gap <= TIE_REL * rng, (
                    f"axis {ax} rank {r}: GPU ray {got[r]} vs oracle ray {ref[r]}, gap {gap:.3e}")
    return same


def lens_slack(problem, b):
    """Oracle bound (per lens parameter) on the lens-gradient change from
    sub-rays within rounding distance of a bilinear cell edge."""
    obs = O.obs_from_problem(problem)
    sl, n, delta = O.cell_edge_slack(problem.lens[b].astype(np.float64), problem.ps[b].astype(np.float64),
                                     problem.latent[b].astype(np.float64), obs, int(problem.n_sub[b]),
                                     problem.geom.tnfw_tau)
    return sl.numpy(), n, delta


def compare(plan, problem, b, res, ref, check_stages=True):
    """Compare sample b of a GPU result with the oracle result `ref`
    (from oracle.loss_grad_problem(..., return_all=True))."""
    from paper_2606_30620_amd import _lib
    out = {}
    loss_g = float(res.loss[b])
    loss_r = float(ref["loss"].detach())
    out["loss"] = abs(loss_g - loss_r) / abs(loss_r)
    assert out["loss"] <= TOL_IMG, ("loss", loss_g, loss_r)
    if res.model is not None:
        out["model"] = relinf(res.model[b].cpu().numpy(), ref["model"].detach().numpy())
        assert out["model"] <= TOL_IMG, ("model", out["model"])
    cm_r = float(ref["chi2_mask"].detach())
    out["chi2_mask"] = abs(float(res.chi2_mask[b]) - cm_r) / max(abs(cm_r), 1e-30)
    assert out["chi2_mask"] <= TOL_IMG
    st = int(res.status[b])
    assert st == ref["status"], ("status", st, ref["status"])
    same_sel = True
    if check_stages:
        tr = ref["transform"]
        if tr is not None:
            kn = plan.debug_fetch(_lib.DBG_KNOTS, b)
            sel = plan.debug_fetch(_lib.DBG_SELECT, b)
            std = plan.debug_fetch(_lib.DBG_STD, b)
            xs, ys = O.pixel_centres(problem.geom.n_img, float(np.float32(problem.geom.pixel_scale)))
            m = torch.as_tensor(problem.mask.reshape(-1).astype(bool))
            lens = torch.as_tensor(problem.lens[b].astype(np.float64))
            bxm, bym = O.ray_shoot(xs[m], ys[m], lens, int(problem.n_sub[b]), problem.geom.tnfw_tau,
                                   getattr(problem.geom, "epl", False))
            same_sel = selection_agrees(sel, tr, [bxm.numpy(), bym.numpy()])
            mu_o = [float(torch.as_tensor(v).detach()) for v in tr["mu"]]
            s_o = float(torch.as_tensor(tr["s"]).detach())
            out["std"] = max(abs(std[0] - float(mu_o[0])), abs(std[1] - float(mu_o[1])), abs(std[2] - s_o) / s_o)
            assert out["std"] < 1e-5, ("std", std, tr["mu"], tr["s"])
            for ax in range(2):
                out[f"X{ax}"] = relinf(kn[ax, 0], tr["X"][ax].detach().numpy())
                out[f"S{ax}"] = relinf(kn[ax, 1], tr["S"][ax].detach().numpy())
                assert out[f"X{ax}"] < 1e-4, (f"knots axis {ax}", out[f"X{ax}"])
                assert out[f"S{ax}"] < 2e-3, (f"slopes axis {ax}", out[f"S{ax}"])
        src = plan.debug_fetch(_lib.DBG_SOURCE, b)
        out["src"] = relinf(src, ref["src"].detach().numpy())
        assert out["src"] <= TOL_IMG, ("source", out["src"])
        u = plan.debug_fetch(_lib.DBG_PREPSF, b)
        out["prepsf"] = relinf(u, ref["u"].detach().numpy())
        assert out["prepsf"] <= TOL_IMG, ("pre-PSF image", out["prepsf"])
    if res.grad_lens is not None:
        # lens vector: mass (7), subhalo slots (4 n_sub_max, of which the
        # first n_sub are active), lens-light Gaussians (6 n_gauss)
        ns = int(problem.n_sub[b])
        g = problem.geom
        base = 8 if getattr(g, "epl", False) else 7
        lo = base + 4 * g.n_sub_max
        act = np.r_[0:base + 4 * ns]
        light = np.r_[lo:lo + 6 * getattr(g, "n_gauss", 0)]
        inact = np.r_[base + 4 * ns:lo]
        out["g_ps"] = relinf(res.grad_ps[b].cpu().numpy(), ref["grad_ps"].numpy())
        out["g_latent"] = relinf(res.grad_latent[b].cpu().numpy(), ref["grad_latent"].numpy())
        assert out["g_ps"] <= TOL_GRAD, ("grad_ps", res.grad_ps[b].cpu().numpy(), ref["grad_ps"].numpy())
        assert out["g_latent"] <= TOL_GRAD, ("grad_latent", out["g_latent"])
        gl_all = res.grad_lens[b].cpu().numpy()
        assert np.all(gl_all[inact] == 0.0), "inactive subhalo gradient slots must be zero"
        if light.size:
            # the lens light does not move rays: its gradient is one group of
            # its own, independent of the order statistics
            out["g_light"] = relinf(gl_all[light], ref["grad_lens"].numpy()[light])
            assert out["g_light"] <= TOL_GRAD, ("grad light", gl_all[light], ref["grad_lens"].numpy()[light])
        gl = gl_all[act]
        ref_l = ref
        if not same_sel:
            # a near-tie ordered the other way: the oracle's gradient for the
            # GPU's order statistics (the loss itself does not depend on it)
            picks = [(sel[ax][0::2], sel[ax][1::2]) for ax in range(2)]
            ref_l = O.loss_grad_problem(problem, b, picks=picks)
            out["picks"] = "GPU order statistics"
        gr = ref_l["grad_lens"].numpy()[act]
        out["g_lens"] = relinf(gl, gr)
        if out["g_lens"] > TOL_GRAD:
            # sub-rays near a cell edge of the bilinear interpolation may take
            # the other side's derivative: allow the oracle's bound, up to
            # SLACK_MAX times the base tolerance
            slack, npk, delta = lens_slack(problem, b)
            scale = np.abs(gr).max()
            out["g_lens_slack"] = float(slack[act].max() / scale)
            say(f"    lens gradient {out['g_lens']:.2e} > {TOL_GRAD:.0e}: cell-edge allowance "
                f"{out['g_lens_slack']:.2e} of the group norm ({npk} sub-ray axes within {delta:.1e} cells of an edge)")
            assert out["g_lens_slack"] <= SLACK_MAX * TOL_GRAD, ("cell-edge allowance too large", out["g_lens_slack"])
            excess = np.abs(gl - gr) - TOL_GRAD * scale - slack[act]
            assert np.all(excess <= 0), ("grad_lens beyond cell-edge slack", gl, gr, slack[act])
    return out
