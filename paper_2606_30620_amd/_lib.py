"""ctypes binding of librtu.so (include/rtu.h).

Argument marshalling only: every numerical step runs in the library's gfx950
kernels.  Device arrays are torch CUDA tensors (their data pointers are passed
through); host arrays are numpy arrays.  If the library has not been built the
import fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtu.so")

RTU_OK = 0
RTU_EINVAL, RTU_ENOMEM, RTU_EBATCH, RTU_EHIP, RTU_ESTATE, RTU_ENOTFOUND = -1, -2, -3, -4, -5, -6
ST_NONFINITE, ST_NONMONOTONE, ST_MASK_SMALL, ST_DOMAIN, ST_SELECT_SLOW = 1, 2, 4, 8, 16
K_NODES = 22
N_LENS_BASE, N_PER_SUB, N_PS, MAX_SUB = 7, 4, 4, 10
DBG_KNOTS, DBG_SELECT, DBG_STD, DBG_SOURCE, DBG_PREPSF = 1, 2, 3, 4, 5


class Geometry(C.Structure):
    _fields_ = [("n_img", C.c_int32), ("supersample", C.c_int32), ("n_src", C.c_int32),
                ("psf_size", C.c_int32), ("n_sub_max", C.c_int32), ("k_nodes", C.c_int32),
                ("pixel_scale", C.c_float), ("tnfw_tau", C.c_float), ("flags", C.c_uint32)]


class RTUError(RuntimeError):
    pass


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_30620_amd.build` "
                          "(the RTU library has no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    P, VP, I32, SZ = C.c_void_p, C.c_void_p, C.c_int32, C.c_size_t
    lib.rtu_n_lens.argtypes = [C.POINTER(Geometry)]
    lib.rtu_n_lens.restype = I32
    lib.rtu_workspace_bytes.argtypes = [C.POINTER(Geometry), I32]
    lib.rtu_workspace_bytes.restype = SZ
    lib.rtu_plan_create.argtypes = [C.POINTER(Geometry), I32, I32, C.POINTER(P)]
    lib.rtu_plan_destroy.argtypes = [P]
    lib.rtu_set_observation.argtypes = [P, VP, VP, VP, VP]
    lib.rtu_masked_count.argtypes = [P]
    lib.rtu_masked_count.restype = I32
    lib.rtu_loss_grad.argtypes = [P, I32] + [VP] * 11 + [VP]
    lib.rtu_debug_fetch.argtypes = [P, I32, I32, VP, SZ, VP]
    lib.rtu_strerror.argtypes = [C.c_int]
    lib.rtu_strerror.restype = C.c_char_p
    for fn in ("rtu_plan_create", "rtu_plan_destroy", "rtu_set_observation", "rtu_loss_grad",
               "rtu_debug_fetch"):
        getattr(lib, fn).restype = C.c_int
    return lib


LIB = _load()


def check(rc: int, what: str = "") -> None:
    if rc != RTU_OK:
        raise RTUError(f"{what}: {LIB.rtu_strerror(rc).decode()} ({rc})")


def make_geometry(n_img, supersample, n_src, psf_size, pixel_scale, n_sub_max=0, tnfw_tau=0.0) -> Geometry:
    return Geometry(int(n_img), int(supersample), int(n_src), int(psf_size), int(n_sub_max), K_NODES,
                    float(pixel_scale), float(tnfw_tau), 0)


def _ptr(t) -> Optional[int]:
    """Device (torch tensor) or host (numpy) data pointer; None stays None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        assert t.flags["C_CONTIGUOUS"]
        return t.ctypes.data
    assert t.is_contiguous(), "tensors passed to the RTU library must be contiguous"
    return t.data_ptr()


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Plan:
    """An rtu_plan: geometry, device workspace for up to max_batch samples."""

    def __init__(self, geom: Geometry, max_batch: int, device: int = 0):
        self.geom = geom
        self.max_batch = int(max_batch)
        self.device = int(device)
        self.n_lens = LIB.rtu_n_lens(C.byref(geom))
        h = C.c_void_p()
        check(LIB.rtu_plan_create(C.byref(geom), self.max_batch, self.device, C.byref(h)), "rtu_plan_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            LIB.rtu_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def masked_count(self) -> int:
        return LIB.rtu_masked_count(self._h)

    def set_observation(self, image, noise_sigma, psf, mask) -> None:
        a = np.ascontiguousarray(image, dtype=np.float32)
        s = np.ascontiguousarray(noise_sigma, dtype=np.float32)
        k = np.ascontiguousarray(psf, dtype=np.float32)
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        n = self.geom.n_img
        assert a.size == n * n and s.size == n * n and m.size == n * n
        assert k.size == self.geom.psf_size ** 2
        check(LIB.rtu_set_observation(self._h, _ptr(a), _ptr(s), _ptr(k), _ptr(m)), "rtu_set_observation")

    def loss_grad(self, lens, ps, latent, n_sub=None, *, loss, status, chi2_mask=None, grad_lens=None,
                  grad_ps=None, grad_latent=None, model=None, stream=None) -> None:
        """Queue one evaluation of the batch on `stream` (default: torch's current)."""
        B = lens.shape[0]
        check(LIB.rtu_loss_grad(self._h, B, _ptr(lens), _ptr(n_sub), _ptr(ps), _ptr(latent), _ptr(loss),
                                _ptr(chi2_mask), _ptr(grad_lens), _ptr(grad_ps), _ptr(grad_latent),
                                _ptr(model), _ptr(status), _stream_ptr(stream)), "rtu_loss_grad")

    def debug_fetch(self, what: int, sample: int, stream=None) -> np.ndarray:
        g = self.geom
        shape, dt = {
            DBG_KNOTS: ((2, 2, K_NODES), np.float32),
            DBG_SELECT: ((2, 2 * K_NODES), np.int32),
            DBG_STD: ((3,), np.float64),
            DBG_SOURCE: ((g.n_src, g.n_src), np.float32),
            DBG_PREPSF: ((g.n_img, g.n_img), np.float32),
        }[what]
        out = np.zeros(shape, dt)
        check(LIB.rtu_debug_fetch(self._h, what, sample, out.ctypes.data, out.nbytes, _stream_ptr(stream)),
              "rtu_debug_fetch")
        return out


def exported_symbols():
    """Names declared in include/rtu.h that the loaded library exports."""
    return [n for n in ("rtu_n_lens", "rtu_workspace_bytes", "rtu_plan_create", "rtu_plan_destroy",
                        "rtu_set_observation", "rtu_masked_count", "rtu_loss_grad", "rtu_debug_fetch",
                        "rtu_strerror") if hasattr(LIB, n)]
