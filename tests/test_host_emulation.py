"""The library's kernels and runtime compiled for the host with
AddressSanitizer (tests/hostemu): every memory access of a full evaluation is
bounds-checked against its buffer, and the outputs are compared with the FP64
oracle at the parity tolerances.  The cases are the ones where out-of-range
indices come from the data: the 24 x 24 image with 52 masked pixels, 3 x 3
sub-rays, a 128 x 128 source in global memory, a rank-two PSF and lens light
(once a GPU memory fault: the quantile selection's target ranks were out of
order for few masked rays); masks of 10 and 52 pixels with both selections;
the allocation-free entry point; a mask large enough for the masked-ray
chunk launch.  CPU only."""
import os
import struct
import subprocess
import tempfile

import numpy as np
import torch
import pytest

from oracle import rtu_oracle as O
from paper_2606_30620_amd import synth
from tests.hostemu import build as hb

TOL_IMG, TOL_GRAD = 1e-4, 1e-3

pytestmark = pytest.mark.skipif(not hb.available(), reason="no host clang++ with AddressSanitizer")


@pytest.fixture(scope="module")
def driver():
    return hb.build()


def _write(p, path):
    g = p.geom
    with open(path, "wb") as f:
        wts = getattr(p, "ray_weights", None)
        f.write(struct.pack("<9i2f", g.n_img, g.supersample, g.n_src, g.psf_size, g.n_sub_max, g.n_gauss,
                            p.batch, p.lens.shape[1], 0 if wts is None else 1, float(np.float32(g.pixel_scale)),
                            float(g.tnfw_tau)))
        for a, dt in ((p.image, np.float32), (p.noise_sigma, np.float32), (p.psf, np.float32), (p.mask, np.uint8),
                      (p.lens, np.float32), (p.ps, np.float32), (p.latent, np.float32), (p.n_sub, np.int32)):
            f.write(np.ascontiguousarray(a, dtype=dt).tobytes())
        if wts is not None:
            f.write(np.ascontiguousarray(wts, dtype=np.float32).tobytes())


def _run(driver, p, mode=0, flags=0):
    g = p.geom
    B, nl, n, N = p.batch, p.lens.shape[1], g.n_src, g.n_img
    with tempfile.TemporaryDirectory() as d:
        fi, fo = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
        _write(p, fi)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
        r = subprocess.run([driver, fi, fo, str(mode), str(flags)], capture_output=True, text=True, timeout=300,
                           env=env)
        assert "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
        assert r.returncode == 0, (r.returncode, r.stderr[-2000:])
        raw = open(fo, "rb").read()
    off = 0

    def take(dt, cnt):
        nonlocal off
        a = np.frombuffer(raw, dtype=dt, count=cnt, offset=off)
        off += a.nbytes
        return a

    out = {"loss": take(np.float64, B), "chi2_mask": take(np.float64, B), "status": take(np.uint32, B),
           "grad_lens": take(np.float32, B * nl).reshape(B, nl), "grad_ps": take(np.float32, B * 4).reshape(B, 4),
           "grad_latent": take(np.float32, B * n * n).reshape(B, n, n),
           "model": take(np.float32, B * N * N).reshape(B, N, N),
           "select": take(np.int32, B * 4 * O.K_NODES).reshape(B, 2, 2 * O.K_NODES),
           "std": take(np.float64, B * 3).reshape(B, 3)}
    assert off == len(raw)
    return out


def _relinf(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    s = np.abs(b).max()
    return np.abs(a - b).max() / s if s > 0 else np.abs(a - b).max()


def _compare(out, p):
    for b in range(p.batch):
        ref = O.loss_grad_problem(p, b)
        assert abs(out["loss"][b] - float(ref["loss"].detach())) <= TOL_IMG * abs(float(ref["loss"].detach()))
        assert _relinf(out["model"][b], ref["model"].detach().numpy()) <= TOL_IMG
        assert int(out["status"][b]) == int(ref["status"])
        assert _relinf(out["grad_ps"][b], ref["grad_ps"].numpy()) <= TOL_GRAD
        assert _relinf(out["grad_latent"][b], ref["grad_latent"].numpy()) <= TOL_GRAD
        ns, g = int(p.n_sub[b]), p.geom
        act = np.r_[0:7 + 4 * ns, 7 + 4 * g.n_sub_max:p.lens.shape[1]]
        assert _relinf(out["grad_lens"][b][act], ref["grad_lens"].numpy()[act]) <= TOL_GRAD


def _case4():
    from tests.test_gpu_parity import _rank_two_psf
    from tests.test_gpu_sweep import _case
    g, rank_two, seed = _case(4)
    p = synth.make_problem("X", batch=2, seed=seed, geom=g)
    assert rank_two and int(p.mask.sum()) == 52
    p.psf = _rank_two_psf(p.psf)
    return p


def _small_mask(npix):
    p = synth.make_problem("C1")
    m = np.zeros_like(p.mask)
    m.reshape(-1)[500:500 + npix] = 1
    p.mask = m
    return p


@pytest.mark.parametrize("mode", [0, 1])
def test_sweep_case_with_52_masked_pixels(driver, mode):
    p = _case4()
    _compare(_run(driver, p, mode=mode), p)


@pytest.mark.parametrize("npix, flags", [(10, 0), (10, 1), (52, 0), (52, 1)])
def test_small_masks_both_selections(driver, npix, flags):
    p = _small_mask(npix)
    _compare(_run(driver, p, flags=flags), p)


@pytest.mark.parametrize("case", ["case4", "mask10", "mask1"])
def test_uniform_grid_mode(driver, case):
    """RTU_GEOM_UNIFORM: the box from the masked rays' extremes and its
    adjoint, on the same data-dependent cases (one masked pixel: the
    degenerate box)."""
    import dataclasses
    p = _case4() if case == "case4" else _small_mask(10 if case == "mask10" else 1)
    p = dataclasses.replace(p, geom=dataclasses.replace(p.geom, uniform=True))
    _compare(_run(driver, p, flags=2), p)


@pytest.mark.parametrize("case", ["c1", "c1-integer", "ragged", "case4", "mask52"])
def test_weighted_grid(driver, case):
    """rtu_set_ray_weights: the stable radix sort and FP64 weight scan of the
    weighted selection (brightness weights, mean 1 over the mask, the faint
    ones zero; or integer weights 1..3).  The selected rays and the weighted
    standardisation are compared with the oracle in every case.  With 52
    masked rays and these weights the smoothed CDF is non-monotone (status
    bit 2, slopes clamped) and so ill-conditioned that the oracle's own
    binary32 rounding model moves the image by 1 % and the binary32 lens
    gradient can overflow: there the loss is compared within twice the
    oracle's own binary32-rounding change, and the run is a bounds check."""
    import dataclasses
    if case == "case4":
        p = _case4()
    elif case == "mask52":
        p = _small_mask(52)
    elif case == "ragged":
        p = synth.make_problem("X", batch=2, seed=7, geom=synth.Geometry(72, 0.06, 3, 16, 9, 1.2))
    else:
        p = synth.make_problem("C1")
    if case == "c1-integer":
        w = np.random.default_rng(3).integers(1, 4, p.mask.shape).astype(np.float64)
    else:
        img = np.abs(p.image.astype(np.float64))
        w = img / img[p.mask.astype(bool)].mean()
        w[w < 0.2] = 0.0
    p = dataclasses.replace(p, ray_weights=w.astype(np.float32))
    out = _run(driver, p)
    for b in range(p.batch):
        ref = O.loss_grad_problem(p, b, want_grad=False, return_all=True)
        tr = ref["transform"]
        for ax in range(2):
            i0, i1 = tr["idx"][ax]
            assert np.array_equal(out["select"][b, ax], np.stack([i0.numpy(), i1.numpy()], 1).reshape(-1))
        std = [float(tr["mu"][0].detach()), float(tr["mu"][1].detach()), float(tr["s"].detach())]
        assert np.allclose(out["std"][b], std, rtol=1e-5, atol=1e-6)
    if case in ("case4", "mask52"):
        obs = O.obs_from_problem(p)
        for b in range(p.batch):
            ref = O.loss_grad_problem(p, b, want_grad=False)
            args = [torch.as_tensor(x[b].astype(np.float64)) for x in (p.lens, p.ps, p.latent)]
            r32 = O.forward(*args, obs, int(p.n_sub[b]), p.geom.tnfw_tau, round32=True)
            # allowance: the loss change under the oracle's binary32 rounding model
            allow = max(TOL_IMG * abs(float(ref["loss"].detach())),
                        2.0 * abs(float(r32["loss"].detach()) - float(ref["loss"].detach())))
            # the clamped slopes make the lens gradient so large that its binary32
            # value may overflow (status bit 1 on top of bit 2)
            assert ref["status"] & O.ST_NONMONOTONE and int(out["status"][b]) & ~O.ST_NONFINITE == int(ref["status"])
            assert abs(out["loss"][b] - float(ref["loss"].detach())) <= allow
    else:
        _compare(out, p)


@pytest.mark.parametrize("case", ["c1", "case4", "subhaloes"])
def test_epl_deflector(driver, case):
    """RTU_GEOM_EPL: the series tables and the complex vector-Jacobian product
    of the elliptical power law in every kernel (slopes around 2.1; lens
    light and a 128 x 128 grid in global memory with case4; two subhaloes)."""
    if case == "c1":
        p = synth.with_epl(synth.make_problem("C1"))
    elif case == "case4":
        p = synth.with_epl(_case4(), slope_mean=2.3)
    else:
        g = synth.Geometry(40, 0.08, 2, 16, 9, 1.0, n_sub_max=2, tnfw_tau=10.0)
        p = synth.with_epl(synth.make_problem("X", batch=2, seed=12, geom=g), slope_mean=1.85)
    _compare(_run(driver, p, flags=4), p)


@pytest.mark.parametrize("case", ["sie", "uniform"])
def test_large_mask_chunked_rays(driver, case):
    """A mask of 8192 rays or more (8281: all but the border of a 93 x 93
    image, a partial last chunk): the masked rays are shot by the chunk
    launch before the selection, which sums the chunks' moments and ranges
    (the uniform grid also their extreme keys)."""
    g = synth.Geometry(93, 0.054, 1, 16, 9, 1.0)
    p = synth.make_problem("X", batch=1, seed=5, geom=g)
    m = np.zeros_like(p.mask)
    m[1:92, 1:92] = 1
    p.mask = m
    assert int(m.sum()) == 8281
    if case == "uniform":
        import dataclasses
        p = dataclasses.replace(p, geom=dataclasses.replace(p.geom, uniform=True))
    _compare(_run(driver, p, flags=2 if case == "uniform" else 0), p)
