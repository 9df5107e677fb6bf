"""Work and footprint accounting for the sampler (host logic only).

Conventions follow the paper's Table IV: a multiply-accumulate counts as two
floating-point operations, a bias addition and a ReLU as one each.  The
MFMA roofline uses the multiply-accumulate part only (bias and ReLU run on
the vector ALUs in the convolution epilogue).
"""
from __future__ import annotations

from typing import Sequence


def conv_macs_per_pixel(channels: Sequence[int], ksize: int = 3) -> int:
    """Multiply-accumulates per output pixel of a stack of ksize x ksize
    convolutions with channel counts channels[0] -> ... -> channels[-1]."""
    return sum(ksize * ksize * a * b for a, b in zip(channels[:-1], channels[1:]))


def denoiser_flops_per_pixel(channels: Sequence[int], ksize: int = 3,
                             elementwise: bool = True) -> int:
    """2 x MACs, plus (elementwise=True) one flop per bias addition on every
    layer and one per ReLU on every layer but the last (Table IV)."""
    f = 2 * conv_macs_per_pixel(channels, ksize)
    if elementwise:
        f += sum(channels[1:]) + sum(channels[1:-1])
    return f


def denoiser_params(channels: Sequence[int], ksize: int = 3, bias: bool = True) -> int:
    p = conv_macs_per_pixel(channels, ksize)
    if bias:
        p += sum(channels[1:])
    return p


def fused_update_bytes_per_pixel(post_burn_in: bool, mask: bool, welford_window: int = 256,
                                 denoiser_handoff: bool = True) -> float:
    """Algorithmic HBM bytes per pixel and iteration of the fused update:
    x read + write (8), y read (4), G hand-off from the denoiser (4),
    mask (1 byte), FP32 Welford mean/M2 read + write (16) after burn-in,
    and the FP64 merge (read 8+8+8 FP32/FP64 pairs, write 16+8) amortised
    over the window."""
    b = 8.0 + 4.0
    if denoiser_handoff:
        b += 4.0
    if mask:
        b += 1.0
    if post_burn_in:
        b += 16.0 + 48.0 / float(welford_window)
    return b
