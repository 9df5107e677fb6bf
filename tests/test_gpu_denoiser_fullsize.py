"""GPU parity of the denoiser itself, at the tilings the sampler runs.

* Every launch of the fused path (first layer inside the first middle
  layer's or pair's kernel, two middle layers per kernel, the last layer's
  partial sums) is checked against the quantisation-emulating FP64 oracle
  started from the GPU's own input activation of that launch (teacher
  forcing), code by code, on images that span several 960-pixel column
  bands of the pair kernels and end in a partial band.
* At the full 1024^2, 4096^2 and 8192^2 sizes, G of the whole-image fused
  path is compared on sampled 32 x 32 regions (corners, block edges, band
  edges, the last partial band) with the oracle's region form.

The networks carry biases U(-0.05, 0.05): with zero biases and spectral norm
0.9 per layer the activations shrink about 3x per layer and G is too small
for relative bars to mean anything.
"""
import numpy as np
import pytest

import oracle.oracle as O
from paper_2511_00870_amd import pnpula as P
from paper_2511_00870_amd import workloads as W

pytestmark = pytest.mark.gpu
BAND = 32 * 30          # column band of the pair kernels' tile order (pixels)


def say(*a):
    print(*a, flush=True)


def _q(v, fmt, scale=1.0):
    return O.quantize_scaled(v, fmt, scale)


def _ulp(v, fmt, scale=1.0):
    """one code step of the format at |v| (after dividing by the scale)"""
    a = np.abs(np.asarray(v, np.float64)) / scale
    e = np.floor(np.log2(np.maximum(a, 1e-300)))
    if fmt == 1:
        return 2.0 ** (np.maximum(e, -126) - 7) * scale
    return 2.0 ** (np.maximum(e, -6) - 3) * scale


# FP32 accumulation slack of one layer's output, relative to the sum of the
# absolute values of its terms (|W| |input| + |b|): the GPU sums 9 F exact
# products (bf16 x bf16 and e4m3 x e4m3 products are exact in FP32) in its own
# order, so its pre-activation value differs from the exact one by a few units
# in the 24th bit of that sum; 1e-5 leaves a wide margin.  (Relative to the
# value itself there is no bound: a sum that cancels to near zero, or a ReLU
# input near zero, carries the absolute error of its terms.)
ACC_REL = 1e-5


def _abs_layer(ws, fmt, net, j):
    """|W_j| as the layer multiplies it (rounded to its format with its
    per-output-channel scales), for propagating error bounds"""
    w = np.asarray(ws[j], np.float64)
    if fmt[j] == 0:
        return np.abs(w)
    s = O.weight_scales(net, j).reshape(-1, 1, 1, 1)
    return np.abs(_q(w / s, fmt[j]) * s)


def _propagate(F, wabs):
    """upper bound of how far a layer's pre-activation output can move when
    its input moves by at most F (per channel and pixel): |W| * F"""
    cout, cin = wabs.shape[:2]
    ch = np.array([cin, cout], np.int32)
    net = O.Net(ch, [wabs], [np.zeros(cout)])
    return O.layers_from(net, F, 0, 1)[0]


def _flip_bound(v, fmt, scale, e):
    """how far the rounded value of v can move when v itself is only known
    within e: one code step (or 2e, when larger) where v lies within e of a
    rounding boundary, zero elsewhere; returns (bound, possibly-flipped).
    The boundaries are the midpoints to the neighbouring codes: the gap away
    from zero is the code's own step, the gap toward zero the step just inside
    its magnitude, which is half as large when the code is a power of two (the
    lower binade's spacing)."""
    q = _q(v, fmt, scale)
    up = _ulp(q, fmt, scale)
    dn = _ulp(q * (1.0 - 2.0 ** -12), fmt, scale)
    sgn = np.where(q < 0, -1.0, 1.0)
    dist = np.minimum(np.abs(v - (q + sgn * up / 2)), np.abs(v - (q - sgn * dn / 2)))
    near = dist <= e
    return np.where(near, np.maximum(up, 2 * e), 0.0), near


def _scales(ch, ws, bs, fmt, x):
    _, amax = O.denoiser_layers(O.Net(ch, ws, bs), x)
    return [float(2.0 ** np.ceil(np.log2(2 * a / 448))) if f == 2 else 1.0
            for a, f in zip(amax, fmt)]


def _ctx(ch, ws, bs, prec, ny, nx, scales, block=None):
    wl = W.make_workload("d", ny, nx, L=5, sigma_k=1.0, sigma=0.02,
                         block=block or max(ny, nx), halo=len(ws), n_layers=len(ws),
                         features=64, precision=prec, iters=1, burn_in=0, seed=5)
    wl.channels, wl.weights, wl.biases = ch, ws, bs
    return P.Context(P.Config.from_workload(
        wl, act_scales=scales if prec == P.PNPULA_FP8_E4M3 else None))


@pytest.mark.parametrize("prec,K", [(P.PNPULA_BF16, 8), (P.PNPULA_FP8_E4M3, 10)])
@pytest.mark.parametrize("shape", [(37, 71), (48, 2000)])
def test_fused_launches_teacher_forced(prec, K, shape):
    """Each launch of the sampler's denoiser path against the emulating
    oracle run from that launch's GPU input (teacher forcing).

    Error model: every layer's GPU value before rounding lies within
    ACC_REL |v| of the exact one, plus what rounding flips of earlier layers
    inside the same launch can add (|W| times one code step at every value
    that sat within its own bound of a rounding boundary).  A stored code
    must equal the exact rounding wherever that bound keeps the value off a
    boundary, and lie within one code step elsewhere; G must lie within its
    bound everywhere.  At most 2e-3 of the stored codes may differ at all."""
    ny, nx = shape
    say(f"case teacher-forced fused launches precision={prec} K={K} {ny}x{nx}")
    ch, ws, bs = W.denoiser_weights(K, 64, seed=61 + K, bias_scale=0.05)
    fmt = W.layer_formats(K, prec)
    x = W.synthetic_image(ny, nx, 71)
    scales = _scales(ch, ws, bs, fmt, x if ny * nx < 10000 else x[:, :256]) \
        if prec == P.PNPULA_FP8_E4M3 else [1.0] * K
    net = O.Net(ch, ws, bs, fmt, scales)
    ctx = _ctx(ch, ws, bs, prec, ny, nx, scales)
    G, stages = ctx.denoise_stages(x.astype(np.float32))
    assert len(stages) >= 2
    inp, k0 = x, 0
    for (k1, act) in stages + [(K - 1, None)]:
        outs = O.layers_from(net, inp, k0, k1 + 1)
        F = None                          # bound on the quantised input's movement
        for j in range(k0, k1 + 1):
            v = outs[j - k0]
            # the layer's input as it multiplies it (rounded to its format)
            prev = inp if j == k0 else outs[j - 1 - k0]
            qin = np.abs(_q(prev, fmt[j], scales[j]))
            if qin.ndim == 2:
                qin = qin[None]
            wabs = _abs_layer(ws, fmt, net, j)
            S = _propagate(qin, wabs) + np.abs(np.asarray(bs[j], np.float64)).reshape(-1, 1, 1)
            e = ACC_REL * S
            if F is not None:
                e = e + _propagate(F, wabs)
            if j < k1:                    # rounded inside the launch
                F, _ = _flip_bound(v, fmt[j + 1], scales[j + 1], e)
        ref = outs[-1]
        if act is None:                   # the last launch: G in FP32
            g = G.astype(np.float64)
            err = np.abs(g - ref[0])
            rel = float(np.linalg.norm(g - ref[0]) / np.linalg.norm(ref[0]))
            say(f"  layers {k0}..{k1} -> G: max err {err.max():.2e}, max bound "
                f"{e.max():.2e} (|G| max {np.abs(ref).max():.2e}), rel {rel:.2e}")
            assert (err <= e[0] + 1e-12).all(), np.argwhere(err > e[0])[:5]
            assert rel <= (5e-3 if prec == P.PNPULA_BF16 else 5e-2)
            break
        f, s = fmt[k1 + 1], scales[k1 + 1]
        refq = _q(ref, f, s)
        bound, near = _flip_bound(ref, f, s, e)
        dev = np.abs(act.astype(np.float64) - refq)
        diff = dev > 0
        bad = dev > bound
        say(f"  layers {k0}..{k1}: {diff.mean():.2e} codes differ, {near.mean():.1e} of the "
            f"values within their bound of a boundary, {int(bad.sum())} outside the bound")
        assert not bad.any(), (np.argwhere(bad)[:5])
        assert diff.mean() <= 2e-3
        inp, k0 = act.astype(np.float64), k1 + 1


def _regions(ny, nx, block):
    rs = [(0, 0), (ny - 32, nx - 32), (block - 16, block - 16), (ny // 2 - 7, 3),
          (ny - 40, nx - 40)]
    for b in range(BAND, nx, BAND):      # band edges and the last (partial) band
        rs.append((min(b // 3, ny - 32), b - 16))
    rs.append((ny // 3, nx - 48 if nx % BAND else nx - 32))
    return rs


@pytest.mark.parametrize("cfgno", [2, 3, 4])
def test_full_size_denoiser_regions(cfgno):
    """G of the whole-image fused path at the configured sizes and tilings,
    on sampled 32 x 32 regions, against the oracle's region form (emulating
    bf16 / e4m3).  Bars: FP32 1e-5; bf16 5e-3 (below one bf16 step, 2^-8);
    e4m3 5e-2 (below one e4m3 step, 2^-4): a wrong tap, channel, scale or
    tile edge gives errors of order one."""
    wl = W.config(cfgno)
    K = wl.n_layers
    ch, ws, bs = W.denoiser_weights(K, 64, seed=7, bias_scale=0.05)
    fmt = W.layer_formats(K, wl.precision) if wl.precision else None
    say(f"case full-size denoiser regions config {cfgno}: {wl.ny}x{wl.nx} precision={wl.precision}")
    rng = np.random.default_rng(cfgno)
    x = np.clip(wl.xbar + 0.03 * rng.standard_normal(wl.xbar.shape), -0.2, 1.2)
    x = x.astype(np.float32)
    scales = None
    if wl.precision == P.PNPULA_FP8_E4M3:
        scales = _scales(ch, ws, bs, fmt, x[:256, :256].astype(np.float64))
    wl.channels, wl.weights, wl.biases = ch, ws, bs
    ctx = P.Context(P.Config.from_workload(wl, act_scales=scales))
    G = ctx.denoise(x)
    del ctx
    net = O.Net(ch, ws, bs, fmt, scales)
    tol = {0: 1e-5, 1: 5e-3, 2: 5e-2}[wl.precision]
    for (y0, x0) in _regions(wl.ny, wl.nx, wl.block_y):
        ref = O.denoise_region(net, x.astype(np.float64), y0, x0, 32, 32)
        e = float(np.linalg.norm(G[y0:y0 + 32, x0:x0 + 32] - ref) / np.linalg.norm(ref))
        say(f"  region ({y0},{x0}) rel {e:.2e}")
        assert e <= tol


def test_step_parity_config2_twenty_sampled_steps():
    """1024^2 FP32 at 20 steps of a running chain (t = 0, 50, ..., 950,
    burn-in and Welford included): the GPU step applied to the GPU's x^(t)
    against the oracle's step from the same x^(t) on sampled regions, with a
    denoiser whose term is visible: the test asserts that (alpha delta/eps) G
    is more than 100x the 1e-5 bar relative to x on every region."""
    wl = W.config(2, bias_scale=0.05)
    say("case 1024^2 FP32, 20 sampled steps")
    ctx = P.Context(P.Config.from_workload(wl))
    oc = O.Chain.from_workload(wl, block=0)
    rng = np.random.default_rng(2)
    worst = 0.0
    t_prev = 0
    for t in range(0, 1000, 50):
        ctx.step(t - t_prev)
        x_t, tt = ctx.get_state()
        assert tt == t
        ctx.step(1)
        t_prev = t + 1
        x1, _ = ctx.get_state()
        for (y0, x0) in [(int(rng.integers(0, wl.ny - 32)), int(rng.integers(0, wl.nx - 32))),
                         (wl.block_y - 16, 2 * wl.block_x - 16)]:
            ref = oc.step_region(x_t.astype(np.float64), t, y0, x0, 32, 32)
            e = float(np.linalg.norm(x1[y0:y0 + 32, x0:x0 + 32] - ref) / np.linalg.norm(ref))
            if t > 0:
                Gr = O.denoise_region(oc.net, x_t.astype(np.float64), y0, x0, 32, 32)
                share = wl.alpha * wl.delta / wl.eps * np.linalg.norm(Gr) / np.linalg.norm(ref)
                assert share > 100 * 1e-5, share
            worst = max(worst, e)
    say(f"  worst per-step rel {worst:.2e}")
    assert worst <= 1e-5
