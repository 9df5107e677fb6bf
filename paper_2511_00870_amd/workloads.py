"""Seeded synthetic workloads for the PnP-ULA sampler.

This module builds *inputs* only: ground-truth images, blur kernels, masks,
observations, denoiser weights, hyper-parameters and serving job streams.  It
contains none of the sampler's arithmetic (no Langevin step, no denoiser
forward pass, no random draws of the chain) and imports nothing from the
product library or from the oracle, so both sides can be fed from it.

Paper context (Sec. III-A, "Application setting"): ground-truth images are
normalised to [0, 1]; observations follow the Gaussian likelihood
y | x ~ N(H x, sigma^2 I) with H a normalised blur and/or a {0,1} diagonal
mask; the chain runs T samples with a 10% burn-in.  The photographs, the
trained denoisers and the motion-blur kernels used in the paper are not
available, so every input here is a seeded synthetic stand-in with the same
structure:

* image: a smooth Gaussian random field (white noise low-passed by a Gaussian
  of correlation length side/32, rescaled to [0.1, 0.6]) plus 8 additive
  constant-intensity rectangles (sides U[side/32, side/8], level U[0, 0.4]),
  clipped to [0, 1];
* blur: an isotropic Gaussian, normalised to unit sum ("normalised blur",
  Sec. III-A2), applied as a same-size linear convolution with zero boundary;
* mask: i.i.d. Bernoulli(p) observed pixels (inpainting, Sec. III-A1);
* noise: y = m * (K xbar + sigma w), w ~ N(0, I);
* denoiser: DnCNN-style residual CNN (Example 2 of Sec. II-B), He-normal
  weights rescaled so that every layer's 3x3 convolution has spectral norm
  0.9 (maximum over a frequency grid of the per-frequency singular value).

Seeds: image s, noise s+1, mask s+2, Philox key s+3, weights 7, with
s = 1000 * config number.
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import List, Optional

import numpy as np

FMT_FP32 = 0
FMT_BF16 = 1
FMT_FP8 = 2
PRECISION_NAMES = {FMT_FP32: "fp32", FMT_BF16: "bf16", FMT_FP8: "fp8_e4m3"}


# --------------------------------------------------------------------------
# images, operators, observations
# --------------------------------------------------------------------------
def gaussian_kernel(L: int, sigma_k: float) -> np.ndarray:
    """L x L isotropic Gaussian k(i,j) ~ exp(-(i^2+j^2)/(2 sigma_k^2)) on
    [-r, r]^2, normalised to unit sum in float64 (odd L)."""
    if L % 2 != 1:
        raise ValueError("blur size must be odd")
    r = L // 2
    t = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-(t[:, None] ** 2 + t[None, :] ** 2) / (2.0 * sigma_k ** 2))
    return g / g.sum()


def synthetic_image(ny: int, nx: int, seed: int) -> np.ndarray:
    """Seeded [0,1] test image: smooth random field + 8 rectangles."""
    rng = np.random.default_rng(seed)
    side = min(ny, nx)
    corr = max(side / 32.0, 1.0)
    white = rng.standard_normal((ny, nx))
    fy = np.fft.fftfreq(ny)[:, None]
    fx = np.fft.rfftfreq(nx)[None, :]
    # Fourier transform of a unit Gaussian of std `corr` (in pixels)
    transfer = np.exp(-2.0 * (math.pi * corr) ** 2 * (fy ** 2 + fx ** 2))
    field = np.fft.irfft2(np.fft.rfft2(white) * transfer, s=(ny, nx))
    lo, hi = field.min(), field.max()
    img = 0.1 + 0.5 * (field - lo) / max(hi - lo, 1e-300)
    for _ in range(8):
        h = int(rng.integers(max(side // 32, 1), max(side // 8, 2) + 1))
        w = int(rng.integers(max(side // 32, 1), max(side // 8, 2) + 1))
        y0 = int(rng.integers(0, max(ny - h, 0) + 1))
        x0 = int(rng.integers(0, max(nx - w, 0) + 1))
        img[y0:y0 + h, x0:x0 + w] += rng.uniform(0.0, 0.4)
    return np.clip(img, 0.0, 1.0)


def bernoulli_mask(ny: int, nx: int, p_observed: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (rng.random((ny, nx)) < p_observed).astype(np.uint8)


def observe(xbar: np.ndarray, kernel: np.ndarray, sigma: float,
            mask: Optional[np.ndarray], seed: int) -> np.ndarray:
    """Synthetic observation y = m * (K xbar + sigma w) (zeros where m = 0).

    K xbar is a same-size linear convolution with zero boundary, evaluated
    with scipy's FFT convolution (data synthesis only)."""
    from scipy.signal import fftconvolve
    rng = np.random.default_rng(seed)
    blurred = fftconvolve(xbar, kernel, mode="same") if kernel.size > 1 else xbar * kernel.item()
    y = blurred + sigma * rng.standard_normal(xbar.shape)
    if mask is not None:
        y = y * mask
    return y


# --------------------------------------------------------------------------
# denoiser weights
# --------------------------------------------------------------------------
def conv_spectral_norm(w: np.ndarray, grid: int = 32) -> float:
    """max over a grid of frequencies of the largest singular value of the
    F_out x F_in symbol W(omega) = sum_taps w[:, :, a, b] exp(-i omega.(a,b)).
    For a zero-padded convolution this bounds the operator norm."""
    fo, fi, kh, kw = w.shape
    om = 2.0 * math.pi * np.arange(grid) / grid
    ey = np.exp(-1j * np.outer(om, np.arange(kh)))  # (grid, kh)
    ex = np.exp(-1j * np.outer(om, np.arange(kw)))  # (grid, kw)
    sym = np.einsum("oiab,ua,vb->uvoi", w.astype(np.complex128), ey, ex)
    sv = np.linalg.svd(sym.reshape(grid * grid, fo, fi), compute_uv=False)
    return float(sv.max())


def denoiser_weights(n_layers: int, features: int, seed: int = 7,
                     spectral: float = 0.9, bias_scale: float = 0.0):
    ch, ws, bs = _denoiser_weights(n_layers, features, seed, spectral, bias_scale)
    return list(ch), [w.copy() for w in ws], [b.copy() for b in bs]


@functools.lru_cache(maxsize=16)
def _denoiser_weights(n_layers: int, features: int, seed: int, spectral: float,
                      bias_scale: float):
    """DnCNN-style layer stack 1 -> F -> ... -> F -> 1 with 3x3 kernels.

    Returns (channels, [w_k (OIHW float32)], [b_k float32]).  He-normal
    init N(0, 2/(9 F_in)), each layer rescaled to spectral norm `spectral`
    (maximum over a 32 x 32 frequency grid).
    Biases are zero unless bias_scale > 0 (then U(-bias_scale, bias_scale)).
    """
    rng = np.random.default_rng(seed)
    ch = [1] + [features] * (n_layers - 1) + [1]
    ws, bs = [], []
    for k in range(n_layers):
        fi, fo = ch[k], ch[k + 1]
        w = rng.standard_normal((fo, fi, 3, 3)) * math.sqrt(2.0 / (9.0 * fi))
        w *= spectral / conv_spectral_norm(w)
        ws.append(w.astype(np.float32))
        if bias_scale > 0:
            bs.append(rng.uniform(-bias_scale, bias_scale, fo).astype(np.float32))
        else:
            bs.append(np.zeros(fo, np.float32))
    return tuple(ch), tuple(ws), tuple(bs)


def wiener_denoiser(a: float = 0.9, sigma_k: float = 1.0):
    """Linear single-layer 'denoiser' G(v) = v - a B3 v, i.e. D = a B3 with
    B3 the normalised 3x3 Gaussian.  With it the PnP-ULA target is Gaussian
    and its moments are available in closed form."""
    b3 = gaussian_kernel(3, sigma_k)
    g = -a * b3
    g[1, 1] += 1.0
    return [1, 1], [g.reshape(1, 1, 3, 3).astype(np.float32)], [np.zeros(1, np.float32)]


# --------------------------------------------------------------------------
# hyper-parameters
# --------------------------------------------------------------------------
def step_size(sigma: float, eps: float, rho: float, n_layers: int,
              alpha: float = 1.0, inv_lambda: float = 0.0, op_norm2: float = 1.0,
              l_eps: Optional[float] = None, frac: float = 0.9) -> float:
    """delta = frac / L with L = ||H||^2 / s2 + alpha L_eps / eps + 1/lambda,
    s2 = sigma^2 (no splitting) or rho (split likelihood).  ||H|| <= 1 for a
    normalised non-negative blur followed by a {0,1} mask, and
    L_eps <= 0.9^K for K layers of spectral norm 0.9 with 1-Lipschitz ReLU."""
    if l_eps is None:
        l_eps = 0.9 ** n_layers
    s2 = rho if rho > 0 else sigma * sigma
    L = op_norm2 / s2 + alpha * l_eps / eps + inv_lambda
    return frac / L


@dataclasses.dataclass
class Workload:
    """Everything a sampler needs, as plain numpy arrays and scalars."""
    name: str
    ny: int
    nx: int
    xbar: np.ndarray
    y: np.ndarray            # float64 observation
    kernel: np.ndarray       # float64 L x L
    mask: Optional[np.ndarray]
    sigma: float
    eps: float
    alpha: float
    delta: float
    rho: float
    inv_lambda: float
    block_y: int
    block_x: int
    halo: int
    channels: List[int]
    weights: List[np.ndarray]
    biases: List[np.ndarray]
    precision: int
    layer_fmt: List[int]
    seed: int
    iters: int
    burn_in: int
    welford_window: int = 256
    # likelihood and splitting variable: 0 Gaussian / 1 Poisson (KL);
    # z-step 0 exact Gaussian draw / 1 PSGLA; operator eta diag(m) K; second
    # block z2 ~ x with the indicator of R+ when rho2 > 0
    likelihood: int = 0
    z_step: int = 0
    eta: float = 0.0
    kappa: float = 0.0
    rho2: float = 0.0
    kappa2: float = 0.0
    # prior: 0 residual CNN (PnP-ULA), 1 TV (PSGLA), 2 DDFB (PnP-ULA)
    prior: int = 0
    beta: float = 0.0
    ddfb_weights: Optional[np.ndarray] = None   # (K, F, 3, 3) float32
    ddfb_gamma: Optional[np.ndarray] = None     # (K,)
    ddfb_thresh: float = 0.0

    @property
    def n_layers(self) -> int:
        return len(self.weights)

    def flat_weights(self) -> np.ndarray:
        return np.concatenate([w.ravel() for w in self.weights]).astype(np.float32)

    def flat_biases(self) -> np.ndarray:
        return np.concatenate([b.ravel() for b in self.biases]).astype(np.float32)


def layer_formats(n_layers: int, precision: int) -> List[int]:
    """Per-layer storage format of each layer's input and weights.
    fp32 and bf16: uniform.  fp8: first and last layer bf16, the rest e4m3."""
    if precision == FMT_FP8:
        return [FMT_BF16] + [FMT_FP8] * (n_layers - 2) + [FMT_BF16]
    return [precision] * n_layers


def make_workload(name: str, ny: int, nx: int, L: int, sigma_k: float, sigma: float,
                  block: int, halo: int, n_layers: int, features: int,
                  precision: int, iters: int, burn_in: int, seed: int,
                  mask_p: Optional[float] = None, split: bool = True,
                  bias_scale: float = 0.0, wiener: bool = False,
                  inv_lambda: float = 0.0) -> Workload:
    xbar = synthetic_image(ny, nx, seed)
    kernel = gaussian_kernel(L, sigma_k)
    mask = bernoulli_mask(ny, nx, mask_p, seed + 2) if mask_p is not None else None
    y = observe(xbar, kernel, sigma, mask, seed + 1)
    if wiener:
        ch, ws, bs = wiener_denoiser()
        l_eps = 1.0
    else:
        ch, ws, bs = denoiser_weights(n_layers, features, 7, 0.9, bias_scale)
        l_eps = None
    eps = sigma * sigma
    rho = sigma * sigma if split else 0.0
    delta = step_size(sigma, eps, rho, len(ws), inv_lambda=inv_lambda, l_eps=l_eps)
    return Workload(name=name, ny=ny, nx=nx, xbar=xbar, y=y, kernel=kernel, mask=mask,
                    sigma=sigma, eps=eps, alpha=1.0, delta=delta, rho=rho,
                    inv_lambda=inv_lambda, block_y=block, block_x=block, halo=halo,
                    channels=ch, weights=ws, biases=bs, precision=precision,
                    layer_fmt=layer_formats(len(ws), precision), seed=seed + 3,
                    iters=iters, burn_in=burn_in)


def config(n: int, **over) -> Workload:
    """The four fixed sampler configurations (1-based), optionally resized
    through keyword overrides (ny, nx, block, iters, ...)."""
    base = {
        1: dict(name="64x64 blur5 K4F16 fp32", ny=64, nx=64, L=5, sigma_k=1.0, sigma=0.01,
                block=64, halo=8, n_layers=4, features=16, precision=FMT_FP32,
                iters=200, burn_in=20),
        2: dict(name="1024x1024 blur9 K8F64 fp32", ny=1024, nx=1024, L=9, sigma_k=2.0,
                sigma=0.02, block=256, halo=8, n_layers=8, features=64,
                precision=FMT_FP32, iters=5000, burn_in=500),
        3: dict(name="4096x4096 blur9 K8F64 bf16", ny=4096, nx=4096, L=9, sigma_k=2.0,
                sigma=0.02, block=512, halo=8, n_layers=8, features=64,
                precision=FMT_BF16, iters=2000, burn_in=200),
        4: dict(name="8192x8192 blur7+mask K10F64 fp8", ny=8192, nx=8192, L=7, sigma_k=1.5,
                sigma=0.01, block=512, halo=12, n_layers=10, features=64,
                precision=FMT_FP8, iters=1000, burn_in=100, mask_p=0.5),
    }[n]
    base.update(over)
    base.setdefault("seed", 1000 * n)
    return make_workload(**base)


# --------------------------------------------------------------------------
# the paper's other applications and priors (Sec. III-A3, III-B)
# --------------------------------------------------------------------------
def motion_blur_kernel(L: int, seed: int, length: Optional[float] = None,
                       substeps: int = 8) -> np.ndarray:
    """Seeded L x L motion-blur kernel (the paper's kernels are not
    available): a random camera trajectory -- a walk whose direction drifts
    with inertia and random turns -- of total length `length` pixels
    (default 0.6 L), centred, rasterised with bilinear splatting and
    normalised to unit sum.  Non-negative, non-separable, sparse."""
    if L % 2 != 1:
        raise ValueError("blur size must be odd")
    rng = np.random.default_rng(seed)
    length = 0.6 * L if length is None else length
    n = max(int(length * substeps), 2)
    ang = rng.uniform(0, 2 * math.pi)
    turn = 0.0
    pts = np.zeros((n, 2))
    for i in range(1, n):
        turn = 0.9 * turn + rng.normal(0, 0.35 / substeps)
        ang += turn
        pts[i] = pts[i - 1] + np.array([math.sin(ang), math.cos(ang)]) / substeps
    pts -= (pts.max(0) + pts.min(0)) / 2           # centre the trajectory
    r = L // 2
    span = np.abs(pts).max()
    if span > r - 1:
        pts *= (r - 1) / span
    k = np.zeros((L, L))
    for (py, px) in pts + r:
        iy, ix = int(math.floor(py)), int(math.floor(px))
        fy, fx = py - iy, px - ix
        for dy, wy in ((0, 1 - fy), (1, fy)):
            for dx, wx in ((0, 1 - fx), (1, fx)):
                k[iy + dy, ix + dx] += wy * wx
    return k / k.sum()


def poisson_workload(name: str, ny: int, nx: int, kernel: np.ndarray, block: int, halo: int,
                     n_layers: int, features: int, precision: int, iters: int, burn_in: int,
                     seed: int, eta: float = 250.0, eps_std: float = 0.05,
                     rho1: float = 10.0, rho2: float = 1e-3, bias_scale: float = 0.0,
                     mask_p: Optional[float] = None) -> Workload:
    """Deconvolution with Poisson noise (Sec. III-A3): y ~ P(eta K xbar), the
    likelihood KL(y || eta K x) on z1 and the indicator of R+ on z2 ~ x, both
    through AXDA and sampled by PSGLA (Sec. III-B1 (ii)): alpha = 1,
    eps = 0.05 (standard deviation), rho1 = 10, rho2 = 1e-3, kappa_i = 0.99
    rho_i, lambda = 0.99 / (4 ||eta H||^2/rho1 + 4/rho2 + 2 alpha L_eps/eps^2),
    gamma = 0.99 / (alpha L_eps/eps^2 + ||eta H||^2/rho1 + 1/rho2 + 1/lambda) / 3,
    with ||H|| <= 1 and L_eps <= 0.9^K."""
    xbar = synthetic_image(ny, nx, seed)
    mask = bernoulli_mask(ny, nx, mask_p, seed + 2) if mask_p is not None else None
    from scipy.signal import fftconvolve
    rng = np.random.default_rng(seed + 1)
    hx = np.maximum(fftconvolve(xbar, kernel, mode="same"), 0.0)
    y = rng.poisson(eta * hx).astype(np.float64)
    if mask is not None:
        y = y * mask
    ch, ws, bs = denoiser_weights(n_layers, features, 7, 0.9, bias_scale)
    alpha, l_eps = 1.0, 0.9 ** n_layers
    eps_var = eps_std ** 2
    nh2 = eta ** 2
    lam = 0.99 / (4 * nh2 / rho1 + 4 / rho2 + 2 * alpha * l_eps / eps_var)
    gamma = 0.99 / (alpha * l_eps / eps_var + nh2 / rho1 + 1 / rho2 + 1 / lam) / 3
    return Workload(name=name, ny=ny, nx=nx, xbar=xbar, y=y, kernel=np.asarray(kernel, np.float64),
                    mask=mask, sigma=1.0, eps=eps_var, alpha=alpha, delta=gamma, rho=rho1,
                    inv_lambda=1.0 / lam, block_y=block, block_x=block, halo=halo, channels=ch,
                    weights=ws, biases=bs, precision=precision,
                    layer_fmt=layer_formats(len(ws), precision),
                    seed=seed + 3, iters=iters, burn_in=burn_in, likelihood=1, z_step=1,
                    eta=eta, kappa=0.99 * rho1, rho2=rho2, kappa2=0.99 * rho2)


def tv_workload(name: str, ny: int, nx: int, kernel: np.ndarray, sigma: float, block: int,
                halo: int, iters: int, burn_in: int, seed: int, beta: float = 40.0,
                rho: float = 1e-5, mask_p: Optional[float] = None) -> Workload:
    """Isotropic TV prior with Gaussian noise (Sec. III-B2 (i)): p = indicator
    of R+, f2 = beta ||.||_{2,1} on z ~ D x through AXDA, x and z sampled by
    PSGLA with rho = 1e-5, beta = 40, gamma = 0.99 (||H||^2/sigma^2 +
    ||D||^2/rho)^-1, kappa = 0.99 rho ||D||^-2, with ||H|| <= 1 and the bound
    ||D||^2 <= 8 of the 2-D forward differences."""
    xbar = synthetic_image(ny, nx, seed)
    mask = bernoulli_mask(ny, nx, mask_p, seed + 2) if mask_p is not None else None
    y = observe(xbar, kernel, sigma, mask, seed + 1)
    d2 = 8.0
    gamma = 0.99 / (1.0 / sigma ** 2 + d2 / rho)
    return Workload(name=name, ny=ny, nx=nx, xbar=xbar, y=y, kernel=np.asarray(kernel, np.float64),
                    mask=mask, sigma=sigma, eps=1.0, alpha=0.0, delta=gamma, rho=rho,
                    inv_lambda=0.0, block_y=block, block_x=block, halo=halo, channels=[1, 1],
                    weights=[np.zeros((1, 1, 3, 3), np.float32)], biases=[np.zeros(1, np.float32)],
                    precision=FMT_FP32, layer_fmt=[FMT_FP32], seed=seed + 3, iters=iters,
                    burn_in=burn_in, kappa=0.99 * rho / d2, prior=1, beta=beta)


def ddfb_params(n_layers: int = 4, features: int = 64, seed: int = 11, thresh: float = 0.05,
                gamma_frac: float = 1.8):
    """Random DDFB parameters (trained weights are not available): K
    weights W_k mapping 1 -> F channels with 3x3 kernels, He-normal then
    rescaled to operator norm 1 (maximum over a frequency grid of the
    per-frequency norm of the F x 1 symbol), step sizes gamma_k = gamma_frac
    / ||W_k||^2 inside (0, 2/||W_k||^2) (Example 3), hard-tanh level thresh."""
    rng = np.random.default_rng(seed)
    ws = []
    for _ in range(n_layers):
        w = rng.standard_normal((features, 1, 3, 3)) * math.sqrt(2.0 / 9.0)
        w /= conv_spectral_norm(w)
        ws.append(w[:, 0].astype(np.float32))
    gam = np.full(n_layers, gamma_frac, np.float64)
    return np.stack(ws), gam, float(thresh)


def ddfb_workload(name: str, ny: int, nx: int, L: int, sigma_k: float, sigma: float,
                  block: int, halo: int, iters: int, burn_in: int, seed: int,
                  n_layers: int = 4, features: int = 64, eps_std: Optional[float] = None,
                  mask_p: Optional[float] = None, split: bool = True) -> Workload:
    """PnP-ULA with the DDFB denoiser (Sec. II-B1 Example 3; Sec. III-B1):
    Gaussian blur (+ optional mask), eps = sigma^2 (variance convention),
    delta = 0.9 / L with L_eps <= 1 (D is firmly nonexpansive in the paper's
    setting; 1 bounds the Lipschitz constant of Id - D used here)."""
    wl = make_workload(name, ny, nx, L=L, sigma_k=sigma_k, sigma=sigma, block=block, halo=halo,
                       n_layers=1, features=1, precision=FMT_FP32, iters=iters, burn_in=burn_in,
                       seed=seed, mask_p=mask_p, split=split)
    w, g, th = ddfb_params(n_layers, features, 11, 0.05 if eps_std is None else eps_std)
    wl.prior = 2
    wl.ddfb_weights, wl.ddfb_gamma, wl.ddfb_thresh = w, g, th
    wl.delta = step_size(wl.sigma, wl.eps, wl.rho, 1, l_eps=1.0)
    return wl


# --------------------------------------------------------------------------
# serving job stream
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Job:
    arrival_s: float
    workload: Workload


def serving_jobs(n_jobs: int = 256, rate: float = 20.0, sides=(256, 512, 1024, 2048),
                 iters=(1000, 5000), seed: int = 5000, n_layers: int = 8,
                 features: int = 64, precision: int = FMT_BF16) -> List[Job]:
    """Poisson arrivals; per job: side, blur size (5/7/9), optional 50% mask,
    sigma ~ U[0.005, 0.05], iteration count ~ U{lo..hi}, eps = sigma^2,
    split rho = sigma^2, tile 256 with halo 8.  All jobs share one denoiser."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += rng.exponential(1.0 / rate)
        side = int(rng.choice(sides))
        L = int(rng.choice([5, 7, 9]))
        masked = bool(rng.random() < 0.5)
        sigma = float(rng.uniform(0.005, 0.05))
        it = int(rng.integers(iters[0], iters[1] + 1))
        wl = make_workload(name=f"job{j}", ny=side, nx=side, L=L, sigma_k=L / 4.5,
                           sigma=sigma, block=min(256, side), halo=8, n_layers=n_layers,
                           features=features, precision=precision, iters=it,
                           burn_in=it // 10, seed=seed + 10 * (j + 1),
                           mask_p=0.5 if masked else None)
        jobs.append(Job(arrival_s=t, workload=wl))
    return jobs
