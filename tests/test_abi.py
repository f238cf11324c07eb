"""The C-ABI library loads and exports every function include/rtu.h declares;
host-side argument validation (no GPU needed)."""
import os
import re

from paper_2606_30620_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "rtu.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rtu_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "rtu_loss_grad" in names and "rtu_plan_create" in names
    for n in names:
        assert hasattr(_lib.LIB, n), n


def test_host_validation_without_gpu():
    L = _lib.LIB
    g = _lib.make_geometry(64, 1, 32, 15, 0.05)
    assert L.rtu_workspace_bytes(g, 1) > 0
    assert L.rtu_n_lens(g) == 7
    bad = _lib.make_geometry(64, 1, 33, 15, 0.05)      # n_src not a power of two
    assert L.rtu_workspace_bytes(bad, 1) == 0
    bad = _lib.make_geometry(64, 1, 32, 14, 0.05)      # even PSF
    assert L.rtu_workspace_bytes(bad, 1) == 0
    bad = _lib.make_geometry(64, 1, 32, 15, 0.05, n_sub_max=_lib.MAX_SUB + 1)
    assert L.rtu_workspace_bytes(bad, 1) == 0
    ok = _lib.make_geometry(64, 1, 32, 15, 0.05, flags=_lib.GEOM_RADIX_SELECT)
    assert L.rtu_workspace_bytes(ok, 1) == L.rtu_workspace_bytes(g, 1)
    uni = _lib.make_geometry(64, 1, 32, 15, 0.05, flags=_lib.GEOM_UNIFORM)
    assert L.rtu_workspace_bytes(uni, 1) == L.rtu_workspace_bytes(g, 1)
    epl = _lib.make_geometry(64, 1, 32, 15, 0.05, flags=_lib.GEOM_EPL)
    assert L.rtu_workspace_bytes(epl, 1) > 0 and L.rtu_n_lens(epl) == 8
    bad = _lib.make_geometry(64, 1, 32, 15, 0.05, flags=8)     # unknown flag
    assert L.rtu_workspace_bytes(bad, 1) == 0
    lit = _lib.make_geometry(64, 1, 32, 15, 0.05, n_sub_max=2, n_gauss=5)
    assert L.rtu_n_lens(lit) == 7 + 4 * 2 + 6 * 5
    bad = _lib.make_geometry(64, 1, 32, 15, 0.05, n_gauss=_lib.MAX_GAUSS + 1)
    assert L.rtu_workspace_bytes(bad, 1) == 0
    assert L.rtu_strerror(_lib.RTU_EBATCH).decode().startswith("batch")
    assert L.rtu_loss_grad(None, 1, *([None] * 12)) == _lib.RTU_EINVAL
