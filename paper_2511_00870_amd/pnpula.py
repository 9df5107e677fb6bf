"""ctypes binding of libpnpula.so (C ABI in include/pnpula.h).

Argument marshalling only: every step of the sampler runs in the HIP
library.  Loading fails loudly when the library has not been built; there is
no fallback path.  Function names mirror the C entry points; the ``Context``
and ``Server`` classes are thin owners of the opaque handles.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpnpula.so")

PNPULA_OK, PNPULA_EINVAL, PNPULA_ENOMEM, PNPULA_EDEVICE, PNPULA_ESTATE, PNPULA_EDIVERGED = \
    0, -1, -2, -3, -4, -5
PNPULA_FP32, PNPULA_BF16, PNPULA_FP8_E4M3 = 0, 1, 2
PNPULA_LIK_GAUSSIAN, PNPULA_LIK_POISSON = 0, 1
PNPULA_PRIOR_CNN, PNPULA_PRIOR_TV, PNPULA_PRIOR_DDFB = 0, 1, 2
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESTATE",
                -5: "EDIVERGED"}

# every symbol include/pnpula.h declares
EXPORTS = [
    "pnpula_create", "pnpula_step", "pnpula_sync", "pnpula_stats", "pnpula_stats_f64",
    "pnpula_get_state", "pnpula_set_state", "pnpula_restore", "pnpula_checkpoint_size",
    "pnpula_checkpoint", "pnpula_resume", "pnpula_get_z", "pnpula_set_z",
    "pnpula_stats_device", "pnpula_data_grad", "pnpula_data_grad_noalloc", "pnpula_denoise",
    "pnpula_denoise_stages",
    "pnpula_calibrate", "pnpula_profile", "pnpula_profile_read", "pnpula_state_device",
    "pnpula_destroy", "pnpula_last_error", "pnpula_create_error", "pnpula_footprint",
    "pnpula_server_create", "pnpula_server_submit", "pnpula_server_tick", "pnpula_server_poll",
    "pnpula_server_result", "pnpula_server_run_until_idle", "pnpula_server_destroy",
    "pnpula_server_last_error",
]


class PnpulaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_fp = C.POINTER(C.c_float)
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u8p = C.POINTER(C.c_uint8)


class pnpula_config(C.Structure):
    _fields_ = [("ny", C.c_int32), ("nx", C.c_int32), ("y", _fp), ("ksize", C.c_int32),
                ("kernel", _fp), ("mask", _u8p), ("sigma", C.c_double), ("eps", C.c_double),
                ("alpha", C.c_double), ("delta", C.c_double), ("rho", C.c_double),
                ("inv_lambda", C.c_double), ("block_y", C.c_int32), ("block_x", C.c_int32),
                ("halo", C.c_int32), ("n_layers", C.c_int32), ("channels", _ip),
                ("weights", _fp), ("biases", _fp), ("precision", C.c_int32),
                ("act_scales", _fp), ("seed", C.c_uint64), ("chain", C.c_uint32),
                ("burn_in", C.c_int32), ("welford_window", C.c_int32), ("x0", _fp),
                ("stream", C.c_void_p), ("likelihood", C.c_int32), ("z_step", C.c_int32),
                ("eta", C.c_double), ("kappa", C.c_double), ("rho2", C.c_double),
                ("kappa2", C.c_double), ("prior", C.c_int32), ("beta", C.c_double),
                ("ddfb_layers", C.c_int32), ("ddfb_features", C.c_int32),
                ("ddfb_weights", _fp), ("ddfb_gamma", _fp), ("ddfb_thresh", C.c_double),
                ("inputs_on_device", C.c_int32)]


_lib = None


def lib():
    """Load libpnpula.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2511_00870_amd.build`")
        # torch ships its own HIP runtime.  Whichever runtime a process loads
        # first serves every later library that asks for it by name, and torch
        # finds no GPU through another build of the runtime: load torch first
        # so that the library and torch share torch's runtime (device tensors
        # and streams then pass between them).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def _declare(L):
    vp = C.c_void_p
    L.pnpula_create.argtypes = [C.POINTER(pnpula_config), C.POINTER(vp)]
    L.pnpula_step.argtypes = [vp, C.c_int32]
    L.pnpula_sync.argtypes = [vp]
    L.pnpula_stats.argtypes = [vp, _fp, _fp, _i64p]
    L.pnpula_stats_f64.argtypes = [vp, _dp, _dp, _i64p]
    L.pnpula_get_state.argtypes = [vp, _fp, _i64p]
    L.pnpula_set_state.argtypes = [vp, _fp, C.c_int64]
    L.pnpula_restore.argtypes = [vp, _fp, C.c_int64, _dp, _dp, C.c_int64]
    L.pnpula_checkpoint_size.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.pnpula_checkpoint.argtypes = [vp, vp, C.c_size_t]
    L.pnpula_resume.argtypes = [vp, vp, C.c_size_t]
    L.pnpula_get_z.argtypes = [vp, _fp, _fp]
    L.pnpula_data_grad.argtypes = [vp, _fp, _fp]
    L.pnpula_data_grad_noalloc.argtypes = [vp, vp, vp]
    L.pnpula_set_z.argtypes = [vp, _fp, _fp]
    L.pnpula_stats_device.argtypes = [vp, vp, vp, _i64p]
    L.pnpula_denoise.argtypes = [vp, _fp, _fp, _fp]
    L.pnpula_denoise_stages.argtypes = [vp, _fp, _fp, _ip, _ip, _fp]
    L.pnpula_calibrate.argtypes = [vp, _fp, _fp]
    L.pnpula_profile.argtypes = [vp, C.c_int32]
    L.pnpula_profile_read.argtypes = [vp, C.c_int32, _dp, _i64p]
    L.pnpula_state_device.argtypes = [vp, C.POINTER(vp), _i64p, _i64p]
    L.pnpula_destroy.argtypes = [vp]
    L.pnpula_destroy.restype = None
    L.pnpula_last_error.argtypes = [vp]
    L.pnpula_last_error.restype = C.c_char_p
    L.pnpula_create_error.restype = C.c_char_p
    L.pnpula_footprint.argtypes = [C.POINTER(pnpula_config), C.POINTER(C.c_size_t)]
    L.pnpula_server_create.argtypes = [C.c_int32, _ip, _fp, _fp, C.c_int32, _fp, C.c_size_t,
                                       C.c_int32, vp, C.POINTER(vp)]
    L.pnpula_server_submit.argtypes = [vp, C.POINTER(pnpula_config), C.c_int32, _i64p]
    L.pnpula_server_tick.argtypes = [vp, _ip]
    L.pnpula_server_poll.argtypes = [vp, C.c_int64, _ip]
    L.pnpula_server_result.argtypes = [vp, C.c_int64, _fp, _fp, _i64p]
    L.pnpula_server_run_until_idle.argtypes = [vp]
    L.pnpula_server_destroy.argtypes = [vp]
    L.pnpula_server_destroy.restype = None
    L.pnpula_server_last_error.argtypes = [vp]
    L.pnpula_server_last_error.restype = C.c_char_p
    for n in EXPORTS:
        f = getattr(L, n)
        if f.restype is C.c_int:   # default
            f.restype = C.c_int


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _fptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_fp)


def _is_device(a) -> bool:
    """a torch tensor on a GPU (torch is imported only when one is passed)"""
    return type(a).__module__.startswith("torch") and getattr(a, "is_cuda", False)


class Config:
    """Owns the arrays a pnpula_config points to."""

    def __init__(self, *, y, kernel, sigma, eps, delta, channels, weights, biases,
                 rho=0.0, alpha=1.0, inv_lambda=0.0, mask=None, block_y=None, block_x=None,
                 halo=0, precision=PNPULA_FP32, act_scales=None, seed=0, chain=0, burn_in=0,
                 welford_window=0, x0=None, stream=None, likelihood=PNPULA_LIK_GAUSSIAN,
                 z_step=0, eta=0.0, kappa=0.0, rho2=0.0, kappa2=0.0, prior=PNPULA_PRIOR_CNN,
                 beta=0.0, ddfb_weights=None, ddfb_gamma=None, ddfb_thresh=0.0):
        """Host arrays (numpy), or torch device tensors for y, kernel, mask
        and x0 together (then inputs_on_device = 1 and the tensors must stay
        alive until the context is created)."""
        dev = _is_device(y)
        if dev:
            ny, nx = (int(v) for v in y.shape)
            self._keep = [v for v in (y, kernel, mask, x0) if v is not None]
            for v in self._keep:
                if not _is_device(v) or not v.is_contiguous():
                    raise ValueError("device inputs: y, kernel, mask and x0 must all be "
                                     "contiguous device tensors")
            ksize = int(kernel.shape[0])
            yp, kp = C.cast(y.data_ptr(), _fp), C.cast(kernel.data_ptr(), _fp)
            mp = None if mask is None else C.cast(mask.data_ptr(), _u8p)
            xp = None if x0 is None else C.cast(x0.data_ptr(), _fp)
        else:
            self.y = _f32(y)
            ny, nx = self.y.shape
            self.kernel = _f32(kernel)
            ksize = self.kernel.shape[0]
            self.mask = None if mask is None else np.ascontiguousarray(mask, np.uint8)
            self.x0 = None if x0 is None else _f32(x0)
            yp, kp = _fptr(self.y), _fptr(self.kernel)
            mp = self.mask.ctypes.data_as(_u8p) if self.mask is not None else None
            xp = _fptr(self.x0)
        self.channels = np.ascontiguousarray(channels, np.int32)
        self.weights = _f32(np.concatenate([np.asarray(w, np.float32).ravel() for w in weights]))
        self.biases = _f32(np.concatenate([np.asarray(b, np.float32).ravel() for b in biases]))
        self.act_scales = None if act_scales is None else _f32(act_scales)
        self.ddfb_weights = None if ddfb_weights is None else _f32(ddfb_weights)
        self.ddfb_gamma = None if ddfb_gamma is None else _f32(ddfb_gamma)
        dK = 0 if self.ddfb_weights is None else int(self.ddfb_weights.shape[0])
        dF = 0 if self.ddfb_weights is None else int(self.ddfb_weights.shape[1])
        self.c = pnpula_config(
            ny, nx, yp, ksize, kp, mp, sigma, eps, alpha, delta, rho, inv_lambda,
            ny if block_y is None else block_y, nx if block_x is None else block_x, halo,
            len(self.channels) - 1, self.channels.ctypes.data_as(_ip), _fptr(self.weights),
            _fptr(self.biases), precision, _fptr(self.act_scales), seed, chain, burn_in,
            welford_window, xp, stream, likelihood, z_step, eta, kappa, rho2, kappa2, prior,
            beta, dK, dF, _fptr(self.ddfb_weights), _fptr(self.ddfb_gamma), ddfb_thresh,
            1 if dev else 0)

    @classmethod
    def from_workload(cls, wl, *, precision=None, act_scales=None, block=None, x0=None,
                      stream=None, chain=0, **over):
        kw = dict(y=wl.y, kernel=wl.kernel, sigma=wl.sigma, eps=wl.eps, delta=wl.delta,
                  rho=wl.rho, alpha=wl.alpha, inv_lambda=wl.inv_lambda, mask=wl.mask,
                  block_y=wl.block_y if block is None else block,
                  block_x=wl.block_x if block is None else block, halo=wl.halo,
                  channels=wl.channels, weights=wl.weights, biases=wl.biases,
                  precision=wl.precision if precision is None else precision,
                  act_scales=act_scales, seed=wl.seed, chain=chain, burn_in=wl.burn_in,
                  welford_window=wl.welford_window, x0=x0, stream=stream,
                  likelihood=wl.likelihood, z_step=wl.z_step, eta=wl.eta, kappa=wl.kappa,
                  rho2=wl.rho2, kappa2=wl.kappa2, prior=wl.prior, beta=wl.beta,
                  ddfb_weights=wl.ddfb_weights, ddfb_gamma=wl.ddfb_gamma,
                  ddfb_thresh=wl.ddfb_thresh)
        kw.update(over)
        return cls(**kw)


def _check(code: int, msg_fn):
    if code != PNPULA_OK:
        raise PnpulaError(code, msg_fn())


class Context:
    """One chain: pnpula_create / step / stats / ... on an opaque handle."""

    def __init__(self, cfg: Config):
        self.cfg = cfg
        self.ny, self.nx = int(cfg.c.ny), int(cfg.c.nx)
        h = C.c_void_p()
        code = lib().pnpula_create(C.byref(cfg.c), C.byref(h))
        _check(code, lambda: lib().pnpula_create_error().decode())
        self.h = h

    def _err(self):
        return lib().pnpula_last_error(self.h).decode()

    def step(self, n: int = 1):
        _check(lib().pnpula_step(self.h, n), self._err)

    def sync(self) -> int:
        code = lib().pnpula_sync(self.h)
        if code not in (PNPULA_OK, PNPULA_EDIVERGED):
            _check(code, self._err)
        return code

    def stats(self):
        mean = np.empty((self.ny, self.nx), np.float32)
        var = np.empty((self.ny, self.nx), np.float32)
        n = C.c_int64()
        _check(lib().pnpula_stats(self.h, _fptr(mean), _fptr(var), C.byref(n)), self._err)
        return mean, var, n.value

    def stats_f64(self):
        mean = np.empty((self.ny, self.nx))
        m2 = np.empty((self.ny, self.nx))
        n = C.c_int64()
        _check(lib().pnpula_stats_f64(self.h, mean.ctypes.data_as(_dp), m2.ctypes.data_as(_dp),
                                      C.byref(n)), self._err)
        return mean, m2, n.value

    def get_state(self):
        x = np.empty((self.ny, self.nx), np.float32)
        t = C.c_int64()
        _check(lib().pnpula_get_state(self.h, _fptr(x), C.byref(t)), self._err)
        return x, t.value

    def set_state(self, x, t: int):
        x = _f32(x)
        _check(lib().pnpula_set_state(self.h, _fptr(x), t), self._err)

    def data_grad(self, x):
        """H^T (H x - y) / sigma^2 of the context's data term at x"""
        x = _f32(x)
        g = np.empty((self.ny, self.nx), np.float32)
        _check(lib().pnpula_data_grad(self.h, _fptr(x), _fptr(g)), self._err)
        return g

    def data_grad_noalloc(self, x, g):
        """pnpula_data_grad_noalloc on torch device tensors x, g (float32,
        ny x nx, contiguous); queued on the context's stream"""
        for v in (x, g):
            if not _is_device(v) or not v.is_contiguous() or v.numel() != self.ny * self.nx:
                raise ValueError("x and g must be contiguous device tensors of ny*nx floats")
        _check(lib().pnpula_data_grad_noalloc(self.h, C.c_void_p(x.data_ptr()),
                                              C.c_void_p(g.data_ptr())), self._err)

    def checkpoint(self) -> bytes:
        """the whole chain state as an opaque byte string"""
        n = C.c_size_t()
        _check(lib().pnpula_checkpoint_size(self.h, C.byref(n)), self._err)
        buf = C.create_string_buffer(n.value)
        _check(lib().pnpula_checkpoint(self.h, buf, n.value), self._err)
        return buf.raw

    def resume(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().pnpula_resume(self.h, buf, len(blob)), self._err)

    def get_z(self):
        """(z1, z2) of a chain that holds its splitting variables (PSGLA, TV)"""
        z1 = np.empty((self.ny, self.nx), np.float32)
        z2 = np.empty((self.ny, self.nx), np.float32)
        _check(lib().pnpula_get_z(self.h, _fptr(z1), _fptr(z2)), self._err)
        return z1, z2

    def set_z(self, z1=None, z2=None):
        z1 = None if z1 is None else _f32(z1)
        z2 = None if z2 is None else _f32(z2)
        _check(lib().pnpula_set_z(self.h, _fptr(z1), _fptr(z2)), self._err)

    def stats_device(self, mean, var):
        """pnpula_stats into torch device tensors (float32, ny x nx each,
        either may be None); returns the sample count"""
        n = C.c_int64()
        for v in (mean, var):
            if v is not None and (not _is_device(v) or not v.is_contiguous() or
                                  v.numel() != self.ny * self.nx):
                raise ValueError("mean / var must be contiguous device tensors of ny*nx floats")
        _check(lib().pnpula_stats_device(
            self.h, None if mean is None else C.c_void_p(mean.data_ptr()),
            None if var is None else C.c_void_p(var.data_ptr()), C.byref(n)), self._err)
        return n.value

    def restore(self, x, t, mean, m2, n):
        x = _f32(x)
        mean = np.ascontiguousarray(mean, np.float64)
        m2 = np.ascontiguousarray(m2, np.float64)
        _check(lib().pnpula_restore(self.h, _fptr(x), t, mean.ctypes.data_as(_dp),
                                    m2.ctypes.data_as(_dp), n), self._err)

    def denoise(self, x, layers: bool = False):
        x = _f32(x)
        G = np.empty((self.ny, self.nx), np.float32)
        lay = None
        if layers:
            ch = [int(c) for c in self.cfg.channels[1:]]
            lay = np.empty(sum(ch) * self.ny * self.nx, np.float32)
        _check(lib().pnpula_denoise(self.h, _fptr(x), _fptr(G), _fptr(lay)), self._err)
        if not layers:
            return G
        out, off = [], 0
        for c in self.cfg.channels[1:]:
            n = int(c) * self.ny * self.nx
            out.append(lay[off:off + n].reshape(int(c), self.ny, self.nx))
            off += n
        return G, out

    def denoise_stages(self, x):
        """The fused denoiser path on x: (G, [(layer, activation (F, ny, nx))]) with one
        entry per launch that wrote an activation to memory."""
        x = _f32(x)
        K = len(self.cfg.channels) - 1
        F = int(self.cfg.channels[1]) if K > 1 else 1
        G = np.empty((self.ny, self.nx), np.float32)
        n = C.c_int32()
        lay = np.zeros(max(K, 1), np.int32)
        acts = np.empty(max(K - 1, 1) * F * self.ny * self.nx, np.float32)
        _check(lib().pnpula_denoise_stages(self.h, _fptr(x), _fptr(G), C.byref(n),
                                           lay.ctypes.data_as(_ip), _fptr(acts)), self._err)
        plane = F * self.ny * self.nx
        return G, [(int(lay[i]), acts[i * plane:(i + 1) * plane].reshape(F, self.ny, self.nx))
                   for i in range(n.value)]

    def calibrate(self, x):
        x = _f32(x)
        amax = np.empty(len(self.cfg.channels) - 1, np.float32)
        _check(lib().pnpula_calibrate(self.h, _fptr(x), _fptr(amax)), self._err)
        return amax

    def profile(self, enable: bool):
        _check(lib().pnpula_profile(self.h, int(enable)), self._err)

    def profile_read(self, cls: int):
        ms = C.c_double()
        n = C.c_int64()
        _check(lib().pnpula_profile_read(self.h, cls, C.byref(ms), C.byref(n)), self._err)
        return ms.value, n.value

    def close(self):
        if getattr(self, "h", None):
            lib().pnpula_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pnpula_footprint(cfg: Config) -> int:
    b = C.c_size_t()
    code = lib().pnpula_footprint(C.byref(cfg.c), C.byref(b))
    _check(code, lambda: lib().pnpula_create_error().decode())
    return b.value


class Server:
    """Continuous-batching server: pnpula_server_* on an opaque handle."""

    def __init__(self, channels, weights, biases, precision=PNPULA_BF16, act_scales=None,
                 hbm_budget: int = 0, max_slots: int = 16, stream=None):
        self.channels = np.ascontiguousarray(channels, np.int32)
        self.weights = _f32(np.concatenate([np.asarray(w, np.float32).ravel() for w in weights]))
        self.biases = _f32(np.concatenate([np.asarray(b, np.float32).ravel() for b in biases]))
        self.act_scales = None if act_scales is None else _f32(act_scales)
        h = C.c_void_p()
        code = lib().pnpula_server_create(len(self.channels) - 1,
                                          self.channels.ctypes.data_as(_ip),
                                          _fptr(self.weights), _fptr(self.biases), precision,
                                          _fptr(self.act_scales), hbm_budget, max_slots, stream,
                                          C.byref(h))
        _check(code, lambda: "server creation failed")
        self.h = h
        self.shapes = {}
        self._cfgs = {}

    def _err(self):
        return lib().pnpula_server_last_error(self.h).decode()

    def submit(self, cfg: Config, n_iters: int) -> int:
        jid = C.c_int64()
        _check(lib().pnpula_server_submit(self.h, C.byref(cfg.c), n_iters, C.byref(jid)),
               self._err)
        self.shapes[jid.value] = (int(cfg.c.ny), int(cfg.c.nx))
        return jid.value

    def tick(self) -> int:
        active = C.c_int32()
        _check(lib().pnpula_server_tick(self.h, C.byref(active)), self._err)
        return active.value

    def poll(self, job_id: int) -> bool:
        d = C.c_int32()
        _check(lib().pnpula_server_poll(self.h, job_id, C.byref(d)), self._err)
        return bool(d.value)

    def result(self, job_id: int):
        ny, nx = self.shapes[job_id]
        mean = np.empty((ny, nx), np.float32)
        var = np.empty((ny, nx), np.float32)
        n = C.c_int64()
        _check(lib().pnpula_server_result(self.h, job_id, _fptr(mean), _fptr(var), C.byref(n)),
               self._err)
        return mean, var, n.value

    def run_until_idle(self):
        _check(lib().pnpula_server_run_until_idle(self.h), self._err)

    def close(self):
        if getattr(self, "h", None):
            lib().pnpula_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
