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
RTU_EINVAL, RTU_ENOMEM, RTU_EBATCH, RTU_EHIP, RTU_ESTATE, RTU_ENOTFOUND, RTU_ETOOBIG = -1, -2, -3, -4, -5, -6, -7
NOALLOC_MAX_BYTES = 64 << 20
ST_NONFINITE, ST_NONMONOTONE, ST_MASK_SMALL, ST_DOMAIN = 1, 2, 4, 8
K_NODES = 22
N_LENS_BASE, N_PER_SUB, N_PS, MAX_SUB = 7, 4, 4, 10
N_PER_GAUSS, MAX_GAUSS = 6, 8
DBG_KNOTS, DBG_SELECT, DBG_STD, DBG_SOURCE, DBG_PREPSF, DBG_ONGRID = 1, 2, 3, 4, 5, 6
STAGES = ("prep", "rays_fwd", "psf_fwd", "psf_adj", "rays_adj", "post", "sample", "adam")


class Geometry(C.Structure):
    _fields_ = [("n_img", C.c_int32), ("supersample", C.c_int32), ("n_src", C.c_int32),
                ("psf_size", C.c_int32), ("n_sub_max", C.c_int32), ("k_nodes", C.c_int32),
                ("pixel_scale", C.c_float), ("tnfw_tau", C.c_float), ("flags", C.c_uint32),
                ("n_gauss", C.c_int32)]


LOG_MASK_WORDS = 3


class FitRequest(C.Structure):
    _fields_ = [("geom", Geometry), ("image", C.c_void_p), ("noise_sigma", C.c_void_p), ("psf", C.c_void_p),
                ("arc_mask", C.c_void_p), ("mu0", C.c_void_p), ("rho0", C.c_void_p), ("samples", C.c_int32),
                ("steps", C.c_int32), ("n_sub", C.c_int32), ("lr", C.c_float), ("seed", C.c_uint64),
                ("log_mask", C.c_uint32 * LOG_MASK_WORDS)]


def log_mask_of(indices) -> "C.Array":
    """Bit mask (RTU_LOG_MASK_WORDS words) of the lens and power-spectrum
    parameters (indices into (lens, ps)) whose guide lives in log space."""
    m = (C.c_uint32 * LOG_MASK_WORDS)()
    for i in indices or ():
        m[i // 32] |= 1 << (i % 32)
    return m


class RTUError(RuntimeError):
    pass


def _load():
    # torch ships its own HIP runtime (libamdhip64.so.7, the same soname as
    # ROCm's).  It must be loaded first so that librtu.so binds to that one copy;
    # loading librtu.so first would bring in a second runtime that torch's
    # kernels then cannot use.
    import torch  # noqa: F401
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
    lib.rtu_set_observation.argtypes = [P, VP, VP, VP, VP, VP]
    lib.rtu_set_ray_weights.argtypes = [P, VP, VP]
    lib.rtu_masked_count.argtypes = [P]
    lib.rtu_masked_count.restype = I32
    lib.rtu_loss_grad.argtypes = [P, I32] + [VP] * 11 + [VP]
    lib.rtu_loss_grad_noalloc.argtypes = [C.POINTER(Geometry), I32] + [VP] * 15 + [VP]
    lib.rtu_loss_grad_noalloc.restype = C.c_int
    lib.rtu_debug_fetch.argtypes = [P, I32, I32, VP, SZ, VP]
    lib.rtu_profile_begin.argtypes = [P, I32, C.c_uint32]
    lib.rtu_profile_end.argtypes = [P, VP, VP]
    lib.rtu_fit_create.argtypes = [P, I32, VP, VP, C.c_float, C.c_uint64, I32, I32, VP, C.POINTER(P)]
    lib.rtu_fit_destroy.argtypes = [P]
    lib.rtu_fit_dim.argtypes = [P]
    lib.rtu_fit_dim.restype = I32
    lib.rtu_fit_step.argtypes = [P, I32, VP, VP]
    lib.rtu_fit_read.argtypes = [P, VP, VP, VP, I32, C.POINTER(I32), VP, VP]
    lib.rtu_fit_last_outputs.argtypes = [P, C.POINTER(VP), C.POINTER(VP)]
    lib.rtu_fit_get_state.argtypes = [P, VP, C.POINTER(I32), VP]
    lib.rtu_fit_samples.argtypes = [P, VP, VP]
    lib.rtu_fit_set_state.argtypes = [P, VP, I32]
    lib.rtu_fleet_create.argtypes = [I32, SZ, I32, I32, C.POINTER(P)]
    lib.rtu_fleet_destroy.argtypes = [P]
    lib.rtu_fleet_request_bytes.argtypes = [C.POINTER(FitRequest)]
    lib.rtu_fleet_request_bytes.restype = SZ
    lib.rtu_fleet_submit.argtypes = [P, C.POINTER(FitRequest), C.POINTER(C.c_int64)]
    lib.rtu_fleet_run.argtypes = [P, I32, VP]
    lib.rtu_fleet_sync.argtypes = [P, VP]
    lib.rtu_fleet_poll.argtypes = [P, VP, I32, C.POINTER(I32)]
    lib.rtu_fleet_result.argtypes = [P, C.c_int64, VP, VP, VP, I32, C.POINTER(I32), C.POINTER(C.c_uint32)]
    lib.rtu_fleet_stats.argtypes = [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(SZ), C.POINTER(C.c_int64)]
    lib.rtu_strerror.argtypes = [C.c_int]
    lib.rtu_strerror.restype = C.c_char_p
    for fn in ("rtu_plan_create", "rtu_plan_destroy", "rtu_set_observation", "rtu_set_ray_weights", "rtu_loss_grad",
               "rtu_debug_fetch", "rtu_profile_begin", "rtu_profile_end", "rtu_fit_create",
               "rtu_fit_destroy", "rtu_fit_step", "rtu_fit_read", "rtu_fit_last_outputs",
               "rtu_fit_get_state", "rtu_fit_set_state", "rtu_fit_samples", "rtu_fleet_create",
               "rtu_fleet_destroy", "rtu_fleet_submit", "rtu_fleet_run", "rtu_fleet_sync", "rtu_fleet_poll",
               "rtu_fleet_result", "rtu_fleet_stats"):
        getattr(lib, fn).restype = C.c_int
    return lib


LIB = _load()


def check(rc: int, what: str = "") -> None:
    if rc != RTU_OK:
        raise RTUError(f"{what}: {LIB.rtu_strerror(rc).decode()} ({rc})")


GEOM_RADIX_SELECT = 1
GEOM_UNIFORM = 2
GEOM_EPL = 4


def make_geometry(n_img, supersample, n_src, psf_size, pixel_scale, n_sub_max=0, tnfw_tau=0.0,
                  flags=0, n_gauss=0) -> Geometry:
    return Geometry(int(n_img), int(supersample), int(n_src), int(psf_size), int(n_sub_max), K_NODES,
                    float(pixel_scale), float(tnfw_tau), int(flags), int(n_gauss))


def _ptr(t) -> Optional[int]:
    """Device (torch tensor) or host (numpy) data pointer; None stays None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        assert t.flags["C_CONTIGUOUS"]
        return t.ctypes.data
    assert t.is_contiguous(), "tensors passed to the RTU library must be contiguous"
    return t.data_ptr()


def _ensure_torch_cuda() -> None:
    """Initialise torch's HIP context before the library's first device call,
    so both share one runtime state (streams are torch's)."""
    import torch
    if torch.cuda.is_available():
        torch.cuda.current_stream()


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
        _ensure_torch_cuda()
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

    def set_observation(self, image, noise_sigma, psf, mask, stream=None) -> None:
        """Queue the observation's upload on `stream` (default: torch's current)."""
        a = np.ascontiguousarray(image, dtype=np.float32)
        s = np.ascontiguousarray(noise_sigma, dtype=np.float32)
        k = np.ascontiguousarray(psf, dtype=np.float32)
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        n = self.geom.n_img
        assert a.size == n * n and s.size == n * n and m.size == n * n
        assert k.size == self.geom.psf_size ** 2
        check(LIB.rtu_set_observation(self._h, _ptr(a), _ptr(s), _ptr(k), _ptr(m), _stream_ptr(stream)),
              "rtu_set_observation")

    def set_ray_weights(self, weights, stream=None) -> None:
        """Per-pixel ray weights of the weighted RTU grid ([n_img, n_img]), or
        None for the unweighted grid; after set_observation."""
        if weights is None:
            check(LIB.rtu_set_ray_weights(self._h, None, _stream_ptr(stream)), "rtu_set_ray_weights")
            return
        w = np.ascontiguousarray(weights, dtype=np.float32)
        assert w.size == self.geom.n_img ** 2
        check(LIB.rtu_set_ray_weights(self._h, _ptr(w), _stream_ptr(stream)), "rtu_set_ray_weights")

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
            DBG_ONGRID: ((1,), np.float64),
        }[what]
        out = np.zeros(shape, dt)
        check(LIB.rtu_debug_fetch(self._h, what, sample, out.ctypes.data, out.nbytes, _stream_ptr(stream)),
              "rtu_debug_fetch")
        return out


    def profile_begin(self, max_calls: int, stages=None) -> None:
        """Time the given stages (names of STAGES; None = all) of the next
        max_calls evaluations or fit steps."""
        mask = 0 if stages is None else sum(1 << STAGES.index(s) for s in stages)
        check(LIB.rtu_profile_begin(self._h, int(max_calls), mask), "rtu_profile_begin")

    def profile_end(self):
        """{stage: (total_ms, launches)} of the recorded evaluations."""
        ms = np.zeros(len(STAGES), np.float64)
        n = np.zeros(len(STAGES), np.int32)
        check(LIB.rtu_profile_end(self._h, ms.ctypes.data, n.ctypes.data), "rtu_profile_end")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(STAGES)}


class Fit:
    """An rtu_fit: Gaussian guide over (lens, ps, latent) with Adam, on a plan."""

    def __init__(self, plan: Plan, samples: int, mu0, rho0, lr=1e-2, seed=0, max_steps=1000, n_sub=0,
                 log_params=None):
        """log_params: lens parameter indices whose guide lives in log space
        (mu0, rho0 of those are of the logarithm)."""
        self.plan = plan
        mu0 = np.ascontiguousarray(mu0, dtype=np.float32)
        rho0 = np.ascontiguousarray(rho0, dtype=np.float32)
        h = C.c_void_p()
        mask = log_mask_of(log_params)
        check(LIB.rtu_fit_create(plan._h, int(samples), mu0.ctypes.data, rho0.ctypes.data, float(lr),
                                 int(seed), int(max_steps), int(n_sub), C.addressof(mask), C.byref(h)),
              "rtu_fit_create")
        self._h = h
        self.dim = LIB.rtu_fit_dim(h)
        assert self.dim == mu0.size
        self.S = int(samples)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            LIB.rtu_fit_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n_steps: int = 1, eps=None, stream=None) -> None:
        check(LIB.rtu_fit_step(self._h, int(n_steps), _ptr(eps), _stream_ptr(stream)), "rtu_fit_step")

    def read(self, stream=None):
        mu = np.zeros(self.dim, np.float32)
        rho = np.zeros(self.dim, np.float32)
        n = C.c_int32()
        check(LIB.rtu_fit_read(self._h, mu.ctypes.data, rho.ctypes.data, None, 0, C.byref(n), None,
                               _stream_ptr(stream)), "rtu_fit_read")
        tr = np.zeros(max(n.value, 1), np.float64)
        check(LIB.rtu_fit_read(self._h, None, None, tr.ctypes.data, n.value, C.byref(n), None,
                               _stream_ptr(stream)), "rtu_fit_read")
        return mu, rho, tr[:n.value]

    def status_acc(self, stream=None) -> int:
        """OR of every sample's status word over every step taken."""
        n = C.c_int32()
        st = C.c_uint32()
        check(LIB.rtu_fit_read(self._h, None, None, None, 0, C.byref(n), C.byref(st), _stream_ptr(stream)),
              "rtu_fit_read")
        return st.value

    def get_state(self, stream=None):
        """(state[6, dim]: mu, rho, m_mu, v_mu, m_rho, v_rho; steps taken)."""
        st = np.zeros((6, self.dim), np.float32)
        n = C.c_int32()
        check(LIB.rtu_fit_get_state(self._h, st.ctypes.data, C.byref(n), _stream_ptr(stream)),
              "rtu_fit_get_state")
        return st, n.value

    def samples(self, stream=None):
        """The last step's samples z[S, dim] (host copy)."""
        z = np.zeros((self.S, self.dim), np.float32)
        check(LIB.rtu_fit_samples(self._h, z.ctypes.data, _stream_ptr(stream)), "rtu_fit_samples")
        return z

    def set_state(self, state, steps: int) -> None:
        st = np.ascontiguousarray(state, dtype=np.float32)
        assert st.shape == (6, self.dim)
        check(LIB.rtu_fit_set_state(self._h, st.ctypes.data, int(steps)), "rtu_fit_set_state")


class Fleet:
    """An rtu_fleet: continuous batching of many fits in shared launches."""

    def __init__(self, hbm_budget: int, max_fits: int = 256, sync_every: int = 4, device: int = 0):
        _ensure_torch_cuda()
        h = C.c_void_p()
        check(LIB.rtu_fleet_create(int(device), int(hbm_budget), int(max_fits), int(sync_every), C.byref(h)),
              "rtu_fleet_create")
        self._h = h
        self._dims = {}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            LIB.rtu_fleet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _request(geom: Geometry, image, sigma, psf, mask, mu0, rho0, samples, steps, n_sub=0, lr=1e-2, seed=0,
                 log_params=None):
        arrs = [np.ascontiguousarray(image, np.float32), np.ascontiguousarray(sigma, np.float32),
                np.ascontiguousarray(psf, np.float32), np.ascontiguousarray(mask, np.uint8),
                np.ascontiguousarray(mu0, np.float32), np.ascontiguousarray(rho0, np.float32)]
        req = FitRequest(geom, *[a.ctypes.data for a in arrs], int(samples), int(steps), int(n_sub), float(lr),
                         int(seed), log_mask_of(log_params))
        return req, arrs

    @staticmethod
    def request_bytes(geom, image, sigma, psf, mask, mu0, rho0, samples, steps, n_sub=0) -> int:
        req, keep = Fleet._request(geom, image, sigma, psf, mask, mu0, rho0, samples, steps, n_sub)
        return LIB.rtu_fleet_request_bytes(C.byref(req))

    def submit(self, geom, image, sigma, psf, mask, mu0, rho0, samples, steps, n_sub=0, lr=1e-2, seed=0,
               log_params=None) -> int:
        req, keep = self._request(geom, image, sigma, psf, mask, mu0, rho0, samples, steps, n_sub, lr, seed,
                                  log_params)
        t = C.c_int64()
        check(LIB.rtu_fleet_submit(self._h, C.byref(req), C.byref(t)), "rtu_fleet_submit")
        self._dims[t.value] = (keep[4].size, int(steps))
        return t.value

    def run(self, rounds: int, stream=None) -> None:
        check(LIB.rtu_fleet_run(self._h, int(rounds), _stream_ptr(stream)), "rtu_fleet_run")

    def sync(self, stream=None) -> None:
        check(LIB.rtu_fleet_sync(self._h, _stream_ptr(stream)), "rtu_fleet_sync")

    def poll(self, max_n: int = 4096):
        buf = np.zeros(max_n, np.int64)
        n = C.c_int32()
        check(LIB.rtu_fleet_poll(self._h, buf.ctypes.data, max_n, C.byref(n)), "rtu_fleet_poll")
        return buf[:n.value].tolist()

    def result(self, ticket: int):
        dim, steps = self._dims.pop(ticket)
        mu = np.zeros(dim, np.float32)
        rho = np.zeros(dim, np.float32)
        tr = np.zeros(steps, np.float64)
        n = C.c_int32()
        st = C.c_uint32()
        check(LIB.rtu_fleet_result(self._h, int(ticket), mu.ctypes.data, rho.ctypes.data, tr.ctypes.data, steps,
                                   C.byref(n), C.byref(st)), "rtu_fleet_result")
        return mu, rho, tr[:n.value], st.value

    def stats(self):
        a, q = C.c_int32(), C.c_int32()
        b = C.c_size_t()
        r = C.c_int64()
        check(LIB.rtu_fleet_stats(self._h, C.byref(a), C.byref(q), C.byref(b), C.byref(r)), "rtu_fleet_stats")
        return {"active": a.value, "queued": q.value, "bytes_in_use": b.value, "rounds": r.value}


def exported_symbols():
    """Names declared in include/rtu.h that the loaded library exports."""
    return [n for n in ("rtu_n_lens", "rtu_workspace_bytes", "rtu_plan_create", "rtu_plan_destroy",
                        "rtu_set_observation", "rtu_set_ray_weights", "rtu_masked_count", "rtu_loss_grad",
                        "rtu_loss_grad_noalloc",
                        "rtu_debug_fetch",
                        "rtu_profile_begin", "rtu_profile_end", "rtu_fit_create", "rtu_fit_destroy",
                        "rtu_fit_dim", "rtu_fit_step", "rtu_fit_read", "rtu_fit_last_outputs",
                        "rtu_fit_get_state", "rtu_fit_set_state", "rtu_fit_samples", "rtu_fleet_create",
                        "rtu_fleet_destroy", "rtu_fleet_request_bytes", "rtu_fleet_submit", "rtu_fleet_run",
                        "rtu_fleet_sync", "rtu_fleet_poll", "rtu_fleet_result", "rtu_fleet_stats",
                        "rtu_strerror") if hasattr(LIB, n)]
