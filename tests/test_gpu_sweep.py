"""Parity with the FP64 oracle over a seeded sweep of small geometries: image
sizes that are not multiples of the ray or PSF tiles, 1-3 sub-rays per axis,
source grids of 8-128 points, PSFs of 1-31 taps (rank one, and rank two for
the matrix-core path), 0-3 subhaloes and 0-3 lens-light Gaussians.  Same
tolerances as the other parity tests (see tests/gpu_helpers.py)."""
import math

import numpy as np
import pytest

from paper_2606_30620_amd import synth
from tests.gpu_helpers import say
from tests.test_gpu_parity import _check, _rank_two_psf

pytestmark = pytest.mark.gpu


def _case(k):
    rng = np.random.default_rng(7000 + k)
    n_img = int(rng.choice([24, 37, 48, 61, 72, 90]))
    ss = int(rng.integers(1, 4))
    n_src = int(rng.choice([8, 16, 32, 64, 128]))
    psf = int(rng.choice([1, 5, 9, 15, 21, 31]))
    n_sub = int(rng.integers(0, 4))
    n_gauss = int(rng.integers(0, 4))
    rank_two = bool(rng.integers(0, 2)) and psf > 1
    pix = 6.2 / n_img
    g = synth.Geometry(n_img, pix, ss, n_src, psf, 2.0 / (2.0 * math.sqrt(2.0 * math.log(2.0))),
                       n_sub_max=n_sub, tnfw_tau=10.0 if n_sub else 0.0, n_gauss=n_gauss)
    return g, rank_two, int(rng.integers(1 << 30))


# Case 4 (24 x 24, 52 masked pixels) once ended its GPU run with a memory
# fault.  The cause, found by running the kernels on the host under
# AddressSanitizer (tests/hostemu): with few masked rays the quantile
# selection's target ranks floor(h_k) + {0, 1} were not in ascending order,
# so a histogram bin appeared in two runs of targets, one run's candidate
# slots in LDS were never written, and an uninitialised key's low word was
# used as a ray index into global memory.  The selection now takes the
# distinct ranks in ascending order.
@pytest.mark.parametrize("k", range(8))
def test_sweep_parity(k):
    g, rank_two, seed = _case(k)
    say(f"[gpu] sweep {k}: {g.n_img}x{g.n_img} ss={g.supersample} n_src={g.n_src} psf={g.psf_size}"
        f"{' rank two' if rank_two else ''} n_sub={g.n_sub_max} n_gauss={g.n_gauss}, batch 2")
    p = synth.make_problem("X", batch=2, seed=seed, geom=g)
    if rank_two:
        p.psf = _rank_two_psf(p.psf)
    _check(p, range(2))
