"""Parity on masks of 8192 rays or more, whose masked rays are shot by a
launch of their own (1024-ray chunks over many workgroups) before the
quantile selection: the plain SIE grid, subhaloes, the EPL deflector, the
uniform grid and the weighted grid, each against the oracle.  The masks
(10944 to 14715 rays) end in a partial chunk."""
import dataclasses

import pytest

from paper_2606_30620_amd import synth
from tests.gpu_helpers import say
from tests.test_gpu_parity import _check
from tests.test_gpu_uniform import _check as _check_uniform
from tests.test_gpu_weighted import _brightness_weights

pytestmark = pytest.mark.gpu

CHUNKED_FROM = 8192   # masks of this many rays or more take the masked-ray launch


def _big(seed, **kw):
    g = synth.Geometry(160, 0.03, 1, 32, 9, 1.0, **kw)
    p = synth.make_problem("X", batch=2, seed=seed, geom=g)
    m = int(p.mask.sum())
    assert m >= CHUNKED_FROM and m % 1024, m
    return p, m


def test_large_mask_sie_and_subhaloes():
    p, m = _big(21)
    say(f"[gpu] large mask: 160x160 ss=1 n_src=32, {m} masked rays, SIE")
    _check(p, range(2))
    p, m = _big(43, n_sub_max=2, tnfw_tau=10.0)
    say(f"[gpu] large mask: 160x160 ss=1 n_src=32, {m} masked rays, SIE + 1 truncated NFW")
    _check(p, range(2))


def test_large_mask_epl():
    p, m = _big(28)
    say(f"[gpu] large mask: EPL, {m} masked rays, slopes around 2.1")
    _check(synth.with_epl(p, slope_mean=2.1), range(2))


def test_large_mask_uniform_grid():
    p, m = _big(23)
    say(f"[gpu] large mask: uniform grid, {m} masked rays")
    _check_uniform(dataclasses.replace(p, geom=dataclasses.replace(p.geom, uniform=True)), [0, 1])


def test_large_mask_weighted_grid():
    p, m = _big(27)
    say(f"[gpu] large mask: weighted grid (brightness weights), {m} masked rays")
    _check(dataclasses.replace(p, ray_weights=_brightness_weights(p)), range(2))
