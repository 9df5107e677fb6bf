"""ctypes binding of the FP64 CPU oracle (liboracle.so) -- test infrastructure.

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module.  It builds liboracle.so from oracle.c with
gcc (IEEE arithmetic: no fast-math, no FMA contraction) and wraps the C entry
points with numpy arrays.  Nothing here depends on the product library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
FMT_EXACT, FMT_BF16, FMT_E4M3 = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (always when force=True)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-Wextra", os.path.join(HERE, "oracle.c"),
               "-o", LIB_PATH + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or (
                os.path.getmtime(LIB_PATH) < os.path.getmtime(os.path.join(HERE, "oracle.c"))):
            build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_u8p = C.POINTER(C.c_uint8)


class OracleNet(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("channels", _ip), ("weights", _dp),
                ("biases", _dp), ("layer_fmt", _ip), ("act_scales", _dp)]


class OracleConfig(C.Structure):
    _fields_ = [("ny", C.c_int32), ("nx", C.c_int32), ("y", _dp), ("ksize", C.c_int32),
                ("kernel", _dp), ("mask", _u8p), ("sigma", C.c_double), ("eps", C.c_double),
                ("alpha", C.c_double), ("delta", C.c_double), ("rho", C.c_double),
                ("inv_lambda", C.c_double), ("block_y", C.c_int32), ("block_x", C.c_int32),
                ("halo", C.c_int32), ("net", OracleNet), ("seed", C.c_uint64),
                ("chain", C.c_uint32), ("burn_in", C.c_int32), ("x0", _dp),
                ("likelihood", C.c_int32), ("z_step", C.c_int32), ("eta", C.c_double),
                ("kappa", C.c_double), ("rho2", C.c_double), ("kappa2", C.c_double),
                ("prior", C.c_int32), ("beta", C.c_double), ("ddfb_layers", C.c_int32),
                ("ddfb_features", C.c_int32), ("ddfb_weights", _dp), ("ddfb_gamma", _dp),
                ("ddfb_thresh", C.c_double)]


def _declare(L):
    L.oracle_create.restype = C.c_void_p
    L.oracle_create.argtypes = [C.POINTER(OracleConfig), C.c_char_p, C.c_int]
    L.oracle_step.argtypes = [C.c_void_p, C.c_int32]
    L.oracle_get_state.argtypes = [C.c_void_p, _dp, C.POINTER(C.c_int64)]
    L.oracle_set_state.argtypes = [C.c_void_p, _dp, C.c_int64]
    L.oracle_stats.argtypes = [C.c_void_p, _dp, _dp, C.POINTER(C.c_int64)]
    L.oracle_record_z.argtypes = [C.c_void_p, C.c_int32]
    L.oracle_last_z.argtypes = [C.c_void_p, _dp]
    L.oracle_destroy.argtypes = [C.c_void_p]
    L.oracle_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
    L.oracle_philox4x64_10.argtypes = [C.POINTER(C.c_uint64)] * 3
    L.oracle_gauss_pair.argtypes = [C.c_uint32, C.c_uint32, _dp, _dp]
    L.oracle_noise.argtypes = [C.c_int32, C.c_int32, C.c_uint64, C.c_uint32, C.c_uint32,
                               _dp, _dp]
    L.oracle_blur.argtypes = [_dp, C.c_int32, C.c_int32, _dp, C.c_int32, _dp]
    L.oracle_blur_adjoint.argtypes = [_dp, C.c_int32, C.c_int32, _dp, C.c_int32, _dp]
    L.oracle_conv3x3.argtypes = [_dp, C.c_int32, C.c_int32, C.c_int32, _dp, _dp, C.c_int32,
                                 C.c_int32, _dp]
    L.oracle_quantize.restype = C.c_double
    L.oracle_quantize.argtypes = [C.c_double, C.c_int32]
    L.oracle_quantize_n.argtypes = [_dp, C.c_int64, C.c_int32, C.c_double, _dp]
    L.oracle_weight_scales.argtypes = [C.POINTER(OracleNet), C.c_int32, _dp]
    L.oracle_denoiser.argtypes = [C.POINTER(OracleNet), _dp, C.c_int32, C.c_int32, C.c_int32,
                                  C.c_int32, C.c_int32, _dp]
    L.oracle_denoise_region.argtypes = [C.POINTER(OracleNet), _dp, C.c_int32, C.c_int32,
                                        C.c_int32, C.c_int32, C.c_int32, C.c_int32, _dp]
    L.oracle_denoiser_layers.argtypes = [C.POINTER(OracleNet), _dp, C.c_int32, C.c_int32,
                                         _dp, _dp]
    L.oracle_layers_from.argtypes = [C.POINTER(OracleNet), _dp, C.c_int32, C.c_int32,
                                     C.c_int32, C.c_int32, _dp, _dp]
    L.oracle_data_grad.argtypes = [C.POINTER(OracleConfig), _dp, C.c_int64, _dp]
    L.oracle_num_threads.restype = C.c_int
    L.oracle_step_region.argtypes = [C.POINTER(OracleConfig), _dp, C.c_int64, C.c_int32,
                                     C.c_int32, C.c_int32, C.c_int32, _dp]
    L.oracle_step_region_z.argtypes = [C.POINTER(OracleConfig), _dp, _dp, _dp, C.c_int64,
                                       C.c_int32, C.c_int32, C.c_int32, C.c_int32, _dp]
    L.oracle_get_z.argtypes = [C.c_void_p, _dp, _dp]
    L.oracle_set_z.argtypes = [C.c_void_p, _dp, _dp]
    L.oracle_ddfb.argtypes = [C.POINTER(OracleConfig), _dp, C.c_int32, C.c_int32, _dp]
    L.oracle_grad2d.argtypes = [_dp, C.c_int32, C.c_int32, _dp, _dp]
    L.oracle_grad2d_adjoint.argtypes = [_dp, _dp, C.c_int32, C.c_int32, _dp]
    L.oracle_prox_kl.restype = C.c_double
    L.oracle_prox_kl.argtypes = [C.c_double, C.c_double, C.c_double]
    L.oracle_prox_gauss.restype = C.c_double
    L.oracle_prox_gauss.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double]
    L.oracle_prox_l21.argtypes = [_dp, _dp, C.c_double]


def _d(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# primitives
# --------------------------------------------------------------------------
def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def philox4x64_10(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    m = (1 << 64) - 1
    c = (C.c_uint64 * 4)(*[int(v) & m for v in ctr])
    k = (C.c_uint64 * 2)(*[int(v) & m for v in key])
    o = (C.c_uint64 * 4)()
    lib().oracle_philox4x64_10(c, k, o)
    return np.array(list(o), dtype=np.uint64)


def gauss_pair(w0: int, w1: int):
    a, b = C.c_double(), C.c_double()
    lib().oracle_gauss_pair(w0, w1, C.byref(a), C.byref(b))
    return a.value, b.value


def noise(ny: int, nx: int, seed: int, t: int, chain: int = 0):
    xi = np.empty((ny, nx)); ze = np.empty((ny, nx))
    lib().oracle_noise(ny, nx, seed, t, chain, _d(xi), _d(ze))
    return xi, ze


def blur(x, k) -> np.ndarray:
    x = _f64(x); k = _f64(k)
    out = np.empty_like(x)
    lib().oracle_blur(_d(x), x.shape[0], x.shape[1], _d(k), k.shape[0], _d(out))
    return out


def blur_adjoint(r, k) -> np.ndarray:
    r = _f64(r); k = _f64(k)
    out = np.empty_like(r)
    lib().oracle_blur_adjoint(_d(r), r.shape[0], r.shape[1], _d(k), k.shape[0], _d(out))
    return out


def conv3x3(inp, w, b, relu: bool) -> np.ndarray:
    inp = _f64(inp); w = _f64(w); b = _f64(b)
    cin, ny, nx = inp.shape
    cout = w.shape[0]
    out = np.empty((cout, ny, nx))
    lib().oracle_conv3x3(_d(inp), cin, ny, nx, _d(w), _d(b), cout, int(relu), _d(out))
    return out


def quantize(v, fmt: int):
    f = lib().oracle_quantize
    return np.vectorize(lambda a: f(float(a), fmt), otypes=[np.float64])(np.asarray(v))


def quantize_scaled(v, fmt: int, scale: float = 1.0):
    """quantize(v / scale) * scale over a whole array (one C call)"""
    v = _f64(v)
    out = np.empty_like(v)
    lib().oracle_quantize_n(_d(v), v.size, fmt, float(scale), _d(out))
    return out


class Net:
    """Denoiser parameters held as contiguous float64 arrays."""

    def __init__(self, channels, weights, biases, layer_fmt=None, act_scales=None):
        self.channels = np.ascontiguousarray(channels, dtype=np.int32)
        self.w = _f64(np.concatenate([np.asarray(w, np.float64).ravel() for w in weights]))
        self.b = _f64(np.concatenate([np.asarray(b, np.float64).ravel() for b in biases]))
        self.fmt = None if layer_fmt is None else np.ascontiguousarray(layer_fmt, np.int32)
        self.scales = None if act_scales is None else _f64(act_scales)
        self.struct = OracleNet(
            len(self.channels) - 1, self.channels.ctypes.data_as(_ip), _d(self.w), _d(self.b),
            self.fmt.ctypes.data_as(_ip) if self.fmt is not None else None,
            _d(self.scales) if self.scales is not None else None)

    @property
    def n_layers(self):
        return len(self.channels) - 1


def weight_scales(net: Net, layer: int) -> np.ndarray:
    out = np.empty(int(net.channels[layer + 1]))
    lib().oracle_weight_scales(C.byref(net.struct), layer, _d(out))
    return out


def denoiser(net: Net, x, block: int = 0, halo: int = 0, block_x: Optional[int] = None):
    x = _f64(x)
    G = np.empty_like(x)
    bx = block if block_x is None else block_x
    rc = lib().oracle_denoiser(C.byref(net.struct), _d(x), x.shape[0], x.shape[1], block, bx,
                               halo, _d(G))
    if rc != 0:
        raise ValueError("halo smaller than the receptive field of the denoiser")
    return G


def grad2d(x):
    """(D_h x, D_v x): forward differences, zero in the last column / row."""
    x = _f64(x)
    dh, dv = np.empty_like(x), np.empty_like(x)
    lib().oracle_grad2d(_d(x), x.shape[0], x.shape[1], _d(dh), _d(dv))
    return dh, dv


def grad2d_adjoint(dh, dv):
    dh, dv = _f64(dh), _f64(dv)
    out = np.empty_like(dh)
    lib().oracle_grad2d_adjoint(_d(dh), _d(dv), dh.shape[0], dh.shape[1], _d(out))
    return out


def prox_kl(v, y, kappa):
    return lib().oracle_prox_kl(float(v), float(y), float(kappa))


def prox_gauss(v, y, sigma, kappa):
    return lib().oracle_prox_gauss(float(v), float(y), float(sigma), float(kappa))


def prox_l21(vh, vv, tau):
    a, b = C.c_double(vh), C.c_double(vv)
    lib().oracle_prox_l21(C.byref(a), C.byref(b), float(tau))
    return a.value, b.value


class Ddfb:
    """DDFB parameters: K layers of 1 -> F 3x3 weights, step sizes, threshold."""

    def __init__(self, weights, gammas, thresh):
        self.w = _f64(np.asarray(weights, np.float64).ravel())
        self.K = len(gammas)
        self.F = self.w.size // (9 * self.K)
        self.g = _f64(gammas)
        self.thresh = float(thresh)

    def fill(self, cfg):
        cfg.prior = 2
        cfg.ddfb_layers, cfg.ddfb_features = self.K, self.F
        cfg.ddfb_weights, cfg.ddfb_gamma = _d(self.w), _d(self.g)
        cfg.ddfb_thresh = self.thresh


def ddfb(params: Ddfb, v) -> np.ndarray:
    """D(v) of the DDFB denoiser on a whole image."""
    v = _f64(v)
    cfg = OracleConfig()
    params.fill(cfg)
    out = np.empty_like(v)
    if lib().oracle_ddfb(C.byref(cfg), _d(v), v.shape[0], v.shape[1], _d(out)) != 0:
        raise ValueError("bad DDFB parameters")
    return out


def denoise_region(net: Net, x, y0: int, x0: int, h: int, w: int) -> np.ndarray:
    """G(x) on the region [y0, y0+h) x [x0, x0+w) of the full image x (cost ~
    region size: the region's K-halo window only)."""
    x = _f64(x)
    out = np.empty((h, w))
    rc = lib().oracle_denoise_region(C.byref(net.struct), _d(x), x.shape[0], x.shape[1], y0, x0,
                                     h, w, _d(out))
    if rc != 0:
        raise ValueError("region outside the image")
    return out


def denoiser_layers(net: Net, x):
    """All layer outputs (list of (C_k, ny, nx) arrays) and per-layer input amax."""
    x = _f64(x)
    ny, nx = x.shape
    sizes = [int(c) * ny * nx for c in net.channels[1:]]
    acts = np.empty(sum(sizes))
    amax = np.empty(net.n_layers)
    lib().oracle_denoiser_layers(C.byref(net.struct), _d(x), ny, nx, _d(acts), _d(amax))
    out, off = [], 0
    for c, s in zip(net.channels[1:], sizes):
        out.append(acts[off:off + s].reshape(int(c), ny, nx))
        off += s
    return out, amax


def layers_from(net: Net, inp, k0: int, k1: int):
    """Outputs of layers k0 .. k1-1 applied to `inp` (layer k0's input,
    (channels[k0], ny, nx)): list of (C, ny, nx) arrays."""
    inp = _f64(inp)
    if inp.ndim == 2:
        inp = inp[None]
    _, ny, nx = inp.shape
    sizes = [int(c) * ny * nx for c in net.channels[k0 + 1:k1 + 1]]
    acts = np.empty(sum(sizes))
    rc = lib().oracle_layers_from(C.byref(net.struct), _d(inp), ny, nx, k0, k1, _d(acts), None)
    if rc != 0:
        raise ValueError("layer range outside the network")
    out, off = [], 0
    for c, s in zip(net.channels[k0 + 1:k1 + 1], sizes):
        out.append(acts[off:off + s].reshape(int(c), ny, nx))
        off += s
    return out


# --------------------------------------------------------------------------
# chain
# --------------------------------------------------------------------------
class Chain:
    """One FP64 PnP-ULA chain (mirrors the product's create/step/stats)."""

    def __init__(self, *, y, kernel, sigma, eps, delta, rho=0.0, alpha=1.0, inv_lambda=0.0,
                 mask=None, block_y=0, block_x=0, halo=0, channels=(1, 1),
                 weights=(np.zeros((1, 1, 3, 3)),), biases=(np.zeros(1),),
                 layer_fmt=None, act_scales=None, seed=0, chain=0, burn_in=0, x0=None,
                 likelihood=0, z_step=0, eta=0.0, kappa=0.0, rho2=0.0, kappa2=0.0,
                 prior=0, beta=0.0, ddfb: Optional[Ddfb] = None):
        self.y = _f64(y)
        self.ny, self.nx = self.y.shape
        self.kernel = _f64(kernel)
        self.mask = None if mask is None else np.ascontiguousarray(mask, np.uint8)
        self.x0 = None if x0 is None else _f64(x0)
        self.net = Net(channels, weights, biases, layer_fmt, act_scales)
        self.ddfb = ddfb
        self.cfg = OracleConfig(
            self.ny, self.nx, _d(self.y), self.kernel.shape[0], _d(self.kernel),
            self.mask.ctypes.data_as(_u8p) if self.mask is not None else None,
            sigma, eps, alpha, delta, rho, inv_lambda, block_y, block_x, halo,
            self.net.struct, seed, chain, burn_in,
            _d(self.x0) if self.x0 is not None else None,
            likelihood, z_step, eta, kappa, rho2, kappa2, prior, beta)
        if ddfb is not None:
            ddfb.fill(self.cfg)
            self.cfg.prior = prior if prior else 2
        err = C.create_string_buffer(256)
        h = lib().oracle_create(C.byref(self.cfg), err, 256)
        if not h:
            raise ValueError(err.value.decode())
        self.h = C.c_void_p(h)

    @classmethod
    def from_workload(cls, wl, *, quantized: bool = False, act_scales=None, chain: int = 0,
                      block: Optional[int] = None, **over):
        kw = dict(y=wl.y, kernel=wl.kernel, sigma=wl.sigma, eps=wl.eps, delta=wl.delta,
                  rho=wl.rho, alpha=wl.alpha, inv_lambda=wl.inv_lambda, mask=wl.mask,
                  block_y=wl.block_y if block is None else block,
                  block_x=wl.block_x if block is None else block, halo=wl.halo,
                  channels=wl.channels, weights=wl.weights, biases=wl.biases,
                  layer_fmt=wl.layer_fmt if quantized else None,
                  act_scales=act_scales, seed=wl.seed, chain=chain, burn_in=wl.burn_in,
                  likelihood=getattr(wl, "likelihood", 0), z_step=getattr(wl, "z_step", 0),
                  eta=getattr(wl, "eta", 0.0), kappa=getattr(wl, "kappa", 0.0),
                  rho2=getattr(wl, "rho2", 0.0), kappa2=getattr(wl, "kappa2", 0.0),
                  prior=getattr(wl, "prior", 0), beta=getattr(wl, "beta", 0.0))
        if getattr(wl, "prior", 0) == 2:
            kw["ddfb"] = Ddfb(wl.ddfb_weights, wl.ddfb_gamma, wl.ddfb_thresh)
        kw.update(over)
        return cls(**kw)

    def step(self, n: int = 1) -> int:
        return lib().oracle_step(self.h, n)

    def get_state(self):
        x = np.empty((self.ny, self.nx)); t = C.c_int64()
        lib().oracle_get_state(self.h, _d(x), C.byref(t))
        return x, t.value

    def set_state(self, x, t: int):
        x = _f64(x)
        lib().oracle_set_state(self.h, _d(x), t)

    def stats(self):
        mean = np.empty((self.ny, self.nx)); m2 = np.empty((self.ny, self.nx))
        n = C.c_int64()
        lib().oracle_stats(self.h, _d(mean), _d(m2), C.byref(n))
        return mean, m2, n.value

    def get_z(self):
        """z^(t) of the PSGLA / TV chains: (z1, z2)."""
        z1 = np.empty((self.ny, self.nx)); z2 = np.empty((self.ny, self.nx))
        lib().oracle_get_z(self.h, _d(z1), _d(z2))
        return z1, z2

    def set_z(self, z1, z2=None):
        z1 = _f64(z1)
        z2 = None if z2 is None else _f64(z2)
        lib().oracle_set_z(self.h, _d(z1), _d(z2) if z2 is not None else None)

    def record_z(self, on: bool = True):
        lib().oracle_record_z(self.h, int(on))

    def last_z(self):
        z = np.empty((self.ny, self.nx))
        lib().oracle_last_z(self.h, _d(z))
        return z

    def data_grad(self, x, t: int):
        x = _f64(x)
        g = np.empty_like(x)
        rc = lib().oracle_data_grad(C.byref(self.cfg), _d(x), t, _d(g))
        if rc != 0:
            raise ValueError("halo smaller than 2r")
        return g

    def step_region(self, x, t: int, y0: int, x0: int, h: int, w: int, z=None):
        """x^(t+1) on a region, from the full x^(t) (and z^(t) = (z1, z2) for
        the PSGLA and TV chains); cost ~ region size."""
        x = _f64(x)
        out = np.empty((h, w))
        z1 = z2 = None
        if z is not None:
            z1 = _f64(z[0])
            z2 = None if z[1] is None else _f64(z[1])
        rc = lib().oracle_step_region_z(C.byref(self.cfg), _d(x),
                                        _d(z1) if z1 is not None else None,
                                        _d(z2) if z2 is not None else None, t, y0, x0, h, w,
                                        _d(out))
        if rc != 0:
            raise ValueError("region outside the image or z missing")
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().oracle_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def num_threads() -> int:
    return lib().oracle_num_threads()
