"""Pins of the FP64 CPU oracle against facts fixed outside the oracle:
library routines (numpy's Philox4x64, rocRAND's Philox4x32 header, scipy's
FFT convolution, torch's float64 conv2d and its bf16/e4m3 casts), closed
forms (adjoint identity, finite differences, Gaussian moments) and the
paper's own statements (blocked == monolithic, Sec. IV-B; Example 1 sizes).
"""
import json
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle.oracle as O
from paper_2511_00870_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------------- Philox
def test_philox4x64_matches_numpy():
    # numpy's Philox (4x64-10) emits block philox(counter + 1, key) first
    for key, ctr in [((0, 0), (0, 0, 0, 0)), ((123, 456), (7, 0, 0, 0)),
                     ((2**64 - 1, 99), (2**64 - 2, 5, 6, 7))]:
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                              counter=np.array(ctr, dtype=np.uint64))
        raw = bg.random_raw(8)
        c = list(ctr)
        for blk in range(2):
            # 256-bit counter increment with carry
            i = 0
            while True:
                c[i] = (c[i] + 1) % 2**64
                if c[i] != 0 or i == 3:
                    break
                i += 1
            ref = O.philox4x64_10(c, key)
            assert [int(v) for v in ref] == [int(v) for v in raw[4 * blk:4 * blk + 4]]


def _rocrand_words(queries):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND host reference")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "rr")
        subprocess.run([hipcc, "-O1", os.path.join(HERE, "golden", "rocrand_philox_ref.cpp"),
                        "-o", exe], check=True, capture_output=True)
        inp = "".join(f"{s} {sub} {off}\n" for s, sub, off in queries)
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True)
    return [[int(v) for v in line.split()] for line in out.stdout.strip().splitlines()]


def test_philox4x32_matches_rocrand_header():
    # rocRAND engine(seed, subsequence, offset): key = seed (lo, hi),
    # counter = (offset/4 lo, offset/4 hi, subsequence lo, subsequence hi)
    rng = np.random.default_rng(3)
    qs = []
    for _ in range(12):
        seed = int(rng.integers(0, 2**63))
        c = [int(v) for v in rng.integers(0, 2**32, 4)]
        sub = c[2] | (c[3] << 32)
        off = 4 * (c[0] | (c[1] << 32))
        qs.append((seed, sub, off % 2**64))
    qs.append((0, 0, 0))
    got = _rocrand_words(qs)
    for (seed, sub, off), ref in zip(qs, got):
        q = off // 4
        ctr = [q & 0xFFFFFFFF, (q >> 32) & 0xFFFFFFFF, sub & 0xFFFFFFFF, sub >> 32]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        assert [int(v) for v in O.philox4x32_10(ctr, key)] == ref


# ------------------------------------------------------------ Box-Muller
def test_box_muller_special_values():
    # u1 = 1 (w0 >> 8 = 2^24 - 1) gives radius 0
    assert O.gauss_pair(0xFFFFFFFF, 12345 << 8) == (0.0, 0.0)
    # u2 = 0: all mass on the cosine branch, radius sqrt(-2 ln u1)
    xi, ze = O.gauss_pair(0, 0)
    assert xi == pytest.approx(np.sqrt(2 * 24 * np.log(2)), rel=1e-15) and ze == 0.0
    # u2 = 1/4: all mass on the sine branch
    xi, ze = O.gauss_pair(0, (1 << 22) << 8)
    assert abs(xi) < 1e-15 and ze == pytest.approx(np.sqrt(2 * 24 * np.log(2)), rel=1e-15)


def test_box_muller_moments_and_ks():
    from scipy import stats
    xi, ze = O.noise(1000, 1000, seed=99, t=3)
    for v in (xi.ravel(), ze.ravel()):
        n = v.size
        assert abs(v.mean()) < 5 / np.sqrt(n)
        assert abs(v.var() - 1) < 5 * np.sqrt(2 / n)
        assert abs(stats.kurtosis(v, fisher=False) - 3) < 5 * np.sqrt(24 / n)
        assert stats.kstest(v[:200000], "norm").pvalue > 1e-4
    # cosine and sine branches are uncorrelated; consecutive pixels too
    assert abs(np.corrcoef(xi.ravel(), ze.ravel())[0, 1]) < 5e-3
    assert abs(np.corrcoef(xi.ravel()[:-1], xi.ravel()[1:])[0, 1]) < 5e-3
    # different t / chain give different streams
    base = O.noise(64, 64, seed=99, t=3)[0]
    assert not np.any(O.noise(64, 64, seed=99, t=4)[0] == base)
    assert not np.any(O.noise(64, 64, seed=99, t=3, chain=1)[0] == base)
    assert not np.any(O.noise(64, 64, seed=100, t=3)[0] == base)


# ----------------------------------------------------------- blur, mask
# 19 .. 129: the large motion blurs (Sec. III-A2); 65 and 129 exceed the
# image, so most taps meet the zero boundary
@pytest.mark.parametrize("L", [1, 3, 5, 9, 19, 65, 129])
def test_blur_matches_fft_convolution(L):
    from scipy.signal import fftconvolve
    rng = np.random.default_rng(L)
    x = rng.random((37, 53))
    k = rng.random((L, L))            # non-symmetric: the flip matters
    if L >= 19:
        k = W.motion_blur_kernel(L, seed=L) + 0.01 * k   # sparse trajectory, no symmetry
    ref = fftconvolve(x, k, mode="same")
    assert np.abs(O.blur(x, k) - ref).max() <= 1e-12 * np.abs(ref).max()
    # adjoint = correlation = convolution with the flipped kernel
    r = rng.standard_normal((37, 53))
    ref_adj = fftconvolve(r, k[::-1, ::-1], mode="same")
    assert np.abs(O.blur_adjoint(r, k) - ref_adj).max() <= 1e-12 * np.abs(ref_adj).max()


def test_adjoint_identity_and_norm():
    rng = np.random.default_rng(1)
    k = W.gaussian_kernel(9, 2.0)
    x = rng.standard_normal((48, 40))
    r = rng.standard_normal((48, 40))
    lhs = np.vdot(O.blur(x, k), r)
    rhs = np.vdot(x, O.blur_adjoint(r, k))
    assert abs(lhs - rhs) <= 1e-13 * np.sqrt(np.vdot(x, x) * np.vdot(r, r))
    # ||K|| <= 1 for a normalised non-negative kernel (power iteration)
    v = rng.standard_normal((48, 40))
    for _ in range(200):
        v = O.blur_adjoint(O.blur(v, k), k)
        lam = np.linalg.norm(v)
        v /= lam
    assert lam <= 1.0 + 1e-12


def test_data_gradient_is_gradient_of_likelihood():
    """g = H^T (H x - y)/sigma^2 equals the finite-difference gradient of
    ||y - H x||^2 / (2 sigma^2) with H = diag(m) K (Eq. (potential_gaussian_likelihood))."""
    wl = W.config(1, ny=24, nx=20, block=64, mask_p=0.6, split=False)
    ch = O.Chain.from_workload(wl, block=0)
    rng = np.random.default_rng(5)
    x = rng.random((24, 20))
    g = ch.data_grad(x, t=0)

    def f(v):
        res = wl.mask * O.blur(v, wl.kernel) - wl.y
        return 0.5 * np.vdot(res, res) / wl.sigma ** 2

    h = 1e-4
    for (i, j) in [(0, 0), (5, 7), (23, 19), (12, 3), (1, 18)]:
        e = np.zeros_like(x)
        e[i, j] = h
        fd = (f(x + e) - f(x - e)) / (2 * h)
        assert fd == pytest.approx(g[i, j], rel=1e-6, abs=1e-6)


def test_split_gradient_at_t0_uses_z_zero():
    """With rho > 0 and z^(0) = 0 the x-gradient is H^T H x / rho, the
    gradient of ||H x||^2/(2 rho) (Eq. (sgs:marginal_x) with z = 0)."""
    wl = W.config(1, ny=16, nx=18, block=64, mask_p=0.5, split=True)
    ch = O.Chain.from_workload(wl, block=0)
    x = np.random.default_rng(2).random((16, 18))
    g = ch.data_grad(x, t=0)
    hx = wl.mask * O.blur(x, wl.kernel)
    ref = O.blur_adjoint(wl.mask * hx, wl.kernel) / wl.rho
    assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()


# ---------------------------------------------------------------- CNN
def test_conv3x3_matches_torch_float64():
    import torch
    rng = np.random.default_rng(2)
    for cin, cout, ny, nx in [(1, 16, 13, 17), (16, 16, 9, 8), (64, 1, 6, 11), (3, 5, 1, 1)]:
        inp = rng.standard_normal((cin, ny, nx))
        w = rng.standard_normal((cout, cin, 3, 3))
        b = rng.standard_normal(cout)
        for relu in (False, True):
            ref = torch.nn.functional.conv2d(torch.tensor(inp)[None], torch.tensor(w),
                                             torch.tensor(b), padding=1)[0]
            if relu:
                ref = torch.relu(ref)
            got = O.conv3x3(inp, w, b, relu)
            assert np.abs(got - ref.numpy()).max() <= 1e-13 * max(1.0, np.abs(got).max())


def test_denoiser_matches_torch_sequence():
    import torch
    ch, ws, bs = W.denoiser_weights(5, 12, seed=3, bias_scale=0.05)
    x = np.random.default_rng(4).random((21, 19))
    net = O.Net(ch, ws, bs)
    v = torch.tensor(x)[None, None]
    for k, (w, b) in enumerate(zip(ws, bs)):
        v = torch.nn.functional.conv2d(v, torch.tensor(w, dtype=torch.float64),
                                       torch.tensor(b, dtype=torch.float64), padding=1)
        if k < len(ws) - 1:
            v = torch.relu(v)
    G = O.denoiser(net, x)
    assert np.abs(G - v[0, 0].numpy()).max() <= 1e-13
    acts, amax = O.denoiser_layers(net, x)
    assert np.array_equal(acts[-1][0], G)
    assert amax[0] == np.abs(x).max()


def test_spectral_norm_scaling():
    """Weights scaled to spectral norm 0.9: ||G(x)-G(x')|| <= 0.9^K ||x-x'||
    (zero biases, ReLU 1-Lipschitz) on random pairs."""
    ch, ws, bs = W.denoiser_weights(4, 16, seed=7)
    net = O.Net(ch, ws, bs)
    rng = np.random.default_rng(0)
    for _ in range(3):
        a, b = rng.random((32, 32)), rng.random((32, 32))
        ratio = np.linalg.norm(O.denoiser(net, a) - O.denoiser(net, b)) / np.linalg.norm(a - b)
        assert ratio <= 0.9 ** 4 * (1 + 1e-9)


# ---------------------------------------------------- quantisation
def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(8)
    v = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        rng.standard_normal(1000) * 1e-39]).astype(np.float32)
    ref = torch.tensor(v).to(torch.bfloat16).to(torch.float64).numpy()
    got = O.quantize(v.astype(np.float64), O.FMT_BF16)
    assert np.array_equal(got, ref)


def test_e4m3_rounding_matches_torch_and_saturates():
    import torch
    codes = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64)
    vals = codes.numpy()
    finite = vals[np.isfinite(vals)]
    # every representable value is a fixed point
    assert np.array_equal(O.quantize(finite, O.FMT_E4M3), finite)
    # random values inside the range round like torch's RNE cast
    rng = np.random.default_rng(9)
    v = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-4, 2.6, 20000)).astype(np.float32)
    v = v[np.abs(v) < 448]
    ref = torch.tensor(v).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(O.quantize(v.astype(np.float64), O.FMT_E4M3), ref)
    # ties go to even: 1.0625 is halfway between 1.0 and 1.125
    assert O.quantize(1.0625, O.FMT_E4M3) == 1.0
    assert O.quantize(1.1875, O.FMT_E4M3) == 1.25
    # saturation instead of overflow
    assert O.quantize(470.0, O.FMT_E4M3) == 448.0
    assert O.quantize(-1e9, O.FMT_E4M3) == -448.0
    assert O.quantize(2.0 ** -10, O.FMT_E4M3) == 0.0          # below half the min subnormal
    assert O.quantize(3 * 2.0 ** -11, O.FMT_E4M3) == 2.0 ** -9  # rounds up to min subnormal


def test_weight_scales_are_powers_of_two_covering_amax():
    ch, ws, bs = W.denoiser_weights(4, 16, seed=7)
    fmt = [1, 2, 2, 1]
    net = O.Net(ch, ws, bs, fmt, [1.0] * 4)
    for k in (1, 2):
        s = O.weight_scales(net, k)
        amax = np.abs(ws[k]).reshape(ws[k].shape[0], -1).max(1)
        assert np.all(amax / s <= 448) and np.all(amax / s > 224)
        assert np.all(np.log2(s) == np.round(np.log2(s)))
    assert np.all(O.weight_scales(net, 0) == 1.0)


# ------------------------------------- blocked == monolithic (Sec. IV-B)
def _chain(wl, block, **kw):
    return O.Chain.from_workload(wl, block=block, **kw)


@pytest.mark.parametrize("split,mask_p", [(False, None), (True, None), (True, 0.5)])
def test_blocked_equals_monolithic_bitwise(split, mask_p):
    """Outputs coincide for any number of blocks (the paper states this up to
    machine precision; with the generator keyed by global pixel the whole
    chain, noise included, is bit-identical)."""
    wl = W.make_workload("t", 45, 38, L=5, sigma_k=1.0, sigma=0.02, block=16, halo=4,
                         n_layers=3, features=6, precision=0, iters=5, burn_in=2,
                         seed=11, mask_p=mask_p, split=split, bias_scale=0.05)
    mono = _chain(wl, block=0)
    blk = _chain(wl, block=16)                      # ragged 45 = 2*16 + 13, 38 = 2*16 + 6
    x0 = np.random.default_rng(1).random((45, 38))
    mono.set_state(x0, 0)
    blk.set_state(x0, 0)
    # operators one by one
    for t in (0, 3):
        assert np.array_equal(mono.data_grad(x0, t), blk.data_grad(x0, t))
    assert np.array_equal(O.denoiser(mono.net, x0), O.denoiser(mono.net, x0, block=16, halo=4))
    assert np.array_equal(O.denoiser(mono.net, x0), O.denoiser(mono.net, x0, block=7, halo=3,
                                                                block_x=13))
    # whole iterations
    mono.step(5)
    blk.step(5)
    a, ta = mono.get_state()
    b, tb = blk.get_state()
    assert ta == tb == 5 and np.array_equal(a, b)
    ma, va, na = mono.stats()
    mb, vb, nb = blk.stats()
    assert na == nb == 3 and np.array_equal(ma, mb) and np.array_equal(va, vb)


def test_blocks_need_the_receptive_field():
    """With biases the activations outside the image must be re-zeroed at
    every layer; a halo smaller than the receptive field is refused."""
    ch, ws, bs = W.denoiser_weights(3, 6, seed=1, bias_scale=0.1)
    net = O.Net(ch, ws, bs)
    x = np.random.default_rng(0).random((20, 20))
    with pytest.raises(ValueError):
        O.denoiser(net, x, block=10, halo=2)
    wl = W.make_workload("t", 20, 20, L=5, sigma_k=1.0, sigma=0.02, block=10, halo=3,
                         n_layers=3, features=6, precision=0, iters=1, burn_in=0, seed=3)
    with pytest.raises(ValueError):
        _chain(wl, block=10)                     # halo 3 < 2r = 4


def test_paper_example1_shapes():
    """Example 1 / Fig. 1: a 3x3 linear convolution of a 20x20 image has a
    22x22 full output; with B = 4 blocks each block needs a ghost region of
    width L - 1 = 2 around it (here: two-sided halo 2r = 2)."""
    g = json.load(open(os.path.join(HERE, "golden", "paper_counts.json")))["fig1_example"]
    from scipy.signal import convolve2d
    x = np.random.default_rng(0).random(tuple(g["image"]))
    k = np.random.default_rng(1).random((g["kernel"], g["kernel"]))
    assert convolve2d(x, k, mode="full").shape == tuple(g["full_output"])
    # same-size form used here, on a 2x2 grid of 10x10 blocks with halo 2
    wl = W.make_workload("ex1", 20, 20, L=3, sigma_k=1.0, sigma=0.05, block=10, halo=2,
                         n_layers=2, features=4, precision=0, iters=1, burn_in=0, seed=4,
                         bias_scale=0.1)
    assert (20 // 10) ** 2 == g["blocks"]
    mono, blk = _chain(wl, block=0), _chain(wl, block=10)
    assert np.array_equal(mono.data_grad(x, 0), blk.data_grad(x, 0))


# ------------------------------------------------------------- Welford
def test_welford_matches_two_pass():
    wl = W.make_workload("w", 12, 10, L=3, sigma_k=1.0, sigma=0.05, block=12, halo=2,
                         n_layers=2, features=4, precision=0, iters=40, burn_in=7, seed=21)
    ch = _chain(wl, block=0)
    samples = []
    for t in range(40):
        ch.step(1)
        x, tt = ch.get_state()
        if tt > wl.burn_in:
            samples.append(x)
    s = np.array(samples)
    mean, m2, n = ch.stats()
    assert n == 33
    assert np.abs(mean - s.mean(0)).max() <= 1e-12 * np.abs(s).max()
    var = m2 / (n - 1)
    ref = s.var(0, ddof=1)
    assert np.abs(var - ref).max() <= 1e-10 * ref.max()


def test_checkpoint_resume_bitwise():
    wl = W.config(1, ny=20, nx=22, block=64)
    a = _chain(wl, block=0)
    a.step(6)
    xa, ta = a.get_state()
    b = _chain(wl, block=0)
    b.step(3)
    xb, tb = b.get_state()
    c = _chain(wl, block=0)
    c.set_state(xb, tb)
    c.step(3)
    xc, tc = c.get_state()
    assert ta == tc == 6 and np.array_equal(xa, xc)


# --------------------------------------------------- paper's counts
def test_table_counts():
    from paper_2511_00870_amd.accounting import denoiser_flops_per_pixel, denoiser_params
    g = json.load(open(os.path.join(HERE, "golden", "paper_counts.json")))
    d = g["dncnn"]
    ch = [d["channels_in"]] + [d["features"]] * (d["layers"] - 1) + [d["channels_in"]]
    assert denoiser_params(ch) == d["params"]
    assert denoiser_flops_per_pixel(ch) == d["flops_per_pixel"]
    assert round(d["params"] * 4 / 2 ** 20, 2) == d["mem_mib"]
    # DDFB: K layers, each a C->F convolution and its adjoint sharing weights,
    # no biases: parameters K*C*F*9, flops 2 convolutions per layer
    for key in ("ddfb4", "ddfb20"):
        d = g[key]
        p = d["layers"] * denoiser_params([d["channels_in"], d["features"]], bias=False)
        assert p == d["params"] and round(p * 4 / 2 ** 20, 2) == d["mem_mib"]
    d = g["ddfb4"]
    assert 2 * d["layers"] * denoiser_flops_per_pixel(
        [d["channels_in"], d["features"]], elementwise=False) == d["flops_per_pixel"]


def test_step_region_equals_full_step_bitwise():
    """The sampled-region step (used to check full-size GPU runs) is the full
    step restricted to the region, bit for bit, at corners, edges and inside."""
    wl = W.config(1, ny=40, nx=50, block=64, mask_p=0.5, bias_scale=0.05)
    ch = O.Chain.from_workload(wl, block=0)
    x = np.random.default_rng(0).random((40, 50))
    ch.set_state(x, 3)
    ch.step(1)
    full, _ = ch.get_state()
    for (y0, x0, h, w) in [(0, 0, 40, 50), (5, 7, 20, 30), (0, 41, 13, 9), (33, 0, 7, 11)]:
        reg = ch.step_region(x, 3, y0, x0, h, w)
        assert np.array_equal(reg, full[y0:y0 + h, x0:x0 + w])
    with pytest.raises(ValueError):
        ch.step_region(x, 3, 35, 0, 10, 10)


# ------------------------------------- quantised layers, composed (Eq. (cnn:convolution))
def _torch_round(t, dtype):
    """Round float64 values to `dtype` (bf16 or e4m3fn) to nearest, ties to
    even, using torch's casts only.  torch converts float64 through float32
    first, which can double-round a float64 value that lies just off a tie
    of the target format; such values are detected (the float32 value is an
    exact tie) and resolved towards the float64 value's side."""
    import torch
    q = t.to(torch.float32)
    base = q.to(dtype).to(torch.float64)
    up = torch.nextafter(q, torch.tensor(float("inf"))).to(dtype).to(torch.float64)
    dn = torch.nextafter(q, torch.tensor(float("-inf"))).to(dtype).to(torch.float64)
    q64 = q.to(torch.float64)
    tie = (up != dn) & ((q64 - dn) == (up - q64))
    fixed = torch.where(t > q64, up, torch.where(t < q64, dn, base))
    return torch.where(tie, fixed, base)


def test_torch_round_helper_single_rounding():
    import torch
    # 1 + 2^-8 is a bf16 tie; a float64 value just above it must round up
    t = torch.tensor([1 + 2 ** -8 + 2 ** -30, 1 + 2 ** -8 - 2 ** -30, 1 + 2 ** -8,
                      1 + 3 * 2 ** -8], dtype=torch.float64)
    got = _torch_round(t, torch.bfloat16).numpy()
    assert list(got) == [1 + 2 ** -7, 1.0, 1.0, 1 + 2 ** -6]
    # the same for e4m3 (step 2^-3 at 1): tie at 1 + 2^-4
    t = torch.tensor([1 + 2 ** -4 + 2 ** -40, 1 + 2 ** -4 - 2 ** -40], dtype=torch.float64)
    assert list(_torch_round(t, torch.float8_e4m3fn).numpy()) == [1.125, 1.0]


@pytest.mark.parametrize("seed", [0, 1])
def test_quantised_denoiser_matches_torch_composition(seed):
    """The oracle's quantisation-emulation mode against a float64 torch
    reference built from torch's own casts: layer k rounds its input divided
    by its activation scale s_a and its weights divided by a per-output-channel
    power-of-two scale s_w to its format, convolves exactly, multiplies by
    s_w s_a, adds the bias and applies ReLU (all but the last layer).  Four
    layers mix bf16 and e4m3, with non-unit power-of-two activation scales."""
    import torch
    ch, ws, bs = W.denoiser_weights(4, 16, seed=40 + seed, bias_scale=0.05)
    fmt = [O.FMT_BF16, O.FMT_E4M3, O.FMT_E4M3, O.FMT_BF16]
    x = W.synthetic_image(23, 29, 50 + seed)
    # activation scales: powers of two from the exact network's input ranges,
    # with the bf16 layers given non-unit scales too (they must ignore them)
    _, amax = O.denoiser_layers(O.Net(ch, ws, bs), x)
    sa = [0.25, float(2.0 ** np.ceil(np.log2(2 * amax[1] / 448))),
          float(2.0 ** np.ceil(np.log2(2 * amax[2] / 448))), 4.0]
    assert sa[1] != 1.0 and sa[2] != 1.0
    acts, _ = O.denoiser_layers(O.Net(ch, ws, bs, fmt, sa), x)
    tdt = {O.FMT_BF16: torch.bfloat16, O.FMT_E4M3: torch.float8_e4m3fn}
    v = torch.tensor(x, dtype=torch.float64)[None, None]
    for k in range(4):
        w = torch.tensor(ws[k], dtype=torch.float64)
        b = torch.tensor(bs[k], dtype=torch.float64)
        if fmt[k] == O.FMT_E4M3:
            amax_w = w.abs().reshape(w.shape[0], -1).max(1).values.numpy()
            s_w = torch.tensor(2.0 ** np.ceil(np.log2(amax_w / 448.0)))
            s_a = sa[k]
        else:
            s_w = torch.ones(w.shape[0], dtype=torch.float64)
            s_a = 1.0
        vq = _torch_round(v / s_a, tdt[fmt[k]])
        wq = _torch_round(w / s_w[:, None, None, None], tdt[fmt[k]])
        v = torch.nn.functional.conv2d(vq, wq, padding=1) * (s_w * s_a)[None, :, None, None] \
            + b[None, :, None, None]
        if k < 3:
            v = torch.relu(v)
        got = acts[k]
        ref = v[0].numpy()
        err = np.abs(got - ref).max()
        assert err <= 1e-13 * max(1.0, np.abs(ref).max()), (k, err)
        v = torch.tensor(got)[None]       # both sides continue from the same values


def test_projection_term_is_moreau_gradient():
    """The term delta/lambda (clip_[0,1](x) - x) of Eq. (sgs_pnp_ula_psgla:pnp_ula)
    is -delta times the gradient of d_C(x)^2 / (2 lambda), C = [0,1]^N: one
    oracle step with H = I, G = 0 and no splitting, minus its data, noise and
    identity parts, against central finite differences of d_C^2/(2 lambda) at
    points below 0, inside [0,1] and above 1."""
    ny, nx = 6, 7
    rng = np.random.default_rng(12)
    x = rng.uniform(-0.8, 1.8, (ny, nx))
    x[0, 0], x[0, 1], x[0, 2] = -0.3, 0.5, 1.4
    y = rng.uniform(0, 1, (ny, nx))
    sigma, delta, inv_lambda, seed, t = 0.1, 1e-3, 37.0, 77, 5
    ch = [1, 4, 1]
    ws = [np.zeros((4, 1, 3, 3), np.float32), np.zeros((1, 4, 3, 3), np.float32)]
    bs = [np.zeros(4, np.float32), np.zeros(1, np.float32)]
    oc = O.Chain(y=y, kernel=np.ones((1, 1)), sigma=sigma, eps=sigma ** 2, delta=delta,
                 inv_lambda=inv_lambda, channels=ch, weights=ws, biases=bs, seed=seed)
    oc.set_state(x, t)
    oc.step(1)
    x1, _ = oc.get_state()
    xi, _ = O.noise(ny, nx, seed, t)
    proj_term = x1 - x + delta * (x - y) / sigma ** 2 - np.sqrt(2 * delta) * xi

    def moreau(v):
        d = v - np.clip(v, 0.0, 1.0)
        return inv_lambda * np.sum(d * d) / 2.0

    h = 1e-5
    for (i, j) in [(0, 0), (0, 1), (0, 2), (3, 4), (5, 6)]:
        e = np.zeros_like(x)
        e[i, j] = h
        fd = (moreau(x + e) - moreau(x - e)) / (2 * h)
        assert proj_term[i, j] == pytest.approx(-delta * fd, rel=1e-6, abs=1e-12)
    assert abs(proj_term[0, 1]) <= 1e-15 and proj_term[0, 0] > 0 and proj_term[0, 2] < 0


def test_denoise_region_equals_full_denoiser_bitwise():
    """The region form of the denoiser (used to check full-size GPU runs) is
    the monolithic denoiser restricted to the region, bit for bit."""
    ch, ws, bs = W.denoiser_weights(4, 8, seed=5, bias_scale=0.05)
    net = O.Net(ch, ws, bs)
    x = np.random.default_rng(3).random((31, 45))
    full = O.denoiser(net, x)
    for (y0, x0, h, w) in [(0, 0, 31, 45), (3, 9, 10, 20), (0, 40, 5, 5), (27, 0, 4, 13)]:
        assert np.array_equal(O.denoise_region(net, x, y0, x0, h, w), full[y0:y0 + h, x0:x0 + w])
    with pytest.raises(ValueError):
        O.denoise_region(net, x, 30, 0, 4, 4)


@pytest.mark.parametrize("quantised", [False, True])
def test_layers_from_continues_the_network_bitwise(quantised):
    """Running layers k0..K-1 from layer k0's input (used to check each fused
    GPU launch from the GPU's own input activation) equals the tail of the
    whole network's layer outputs, bit for bit."""
    ch, ws, bs = W.denoiser_weights(5, 8, seed=9, bias_scale=0.05)
    fmt = [1, 2, 2, 2, 1] if quantised else None
    sc = [1.0, 2.0 ** -6, 2.0 ** -7, 2.0 ** -7, 1.0] if quantised else None
    net = O.Net(ch, ws, bs, fmt, sc)
    x = np.random.default_rng(8).random((17, 22))
    acts, _ = O.denoiser_layers(net, x)
    assert all(np.array_equal(a, b) for a, b in zip(O.layers_from(net, x, 0, 5), acts))
    for k0 in (1, 3):
        tail = O.layers_from(net, acts[k0 - 1], k0, 5)
        assert all(np.array_equal(a, b) for a, b in zip(tail, acts[k0:]))
    with pytest.raises(ValueError):
        O.layers_from(net, x, 3, 2)
