"""Host-side checks of the C ABI (no GPU compute): the library loads, exports
every function include/pnpula.h declares, and rejects invalid configurations
before touching a device."""
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2511_00870_amd import pnpula as P
from paper_2511_00870_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "pnpula.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pnpula_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _header_functions()
    assert len(names) >= 20
    assert sorted(P.EXPORTS) == names
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (pnpula_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = P.lib()
    for n in names:
        assert hasattr(L, n)


def _cfg(**over):
    wl = W.config(1, ny=40, nx=36, block=16)
    return P.Config.from_workload(wl, **over)


@pytest.mark.parametrize("over,needle", [
    (dict(kernel=np.ones((4, 4)) / 16), "odd"),
    (dict(kernel=np.ones((131, 131)) / 131 ** 2), "odd"),
    (dict(likelihood=P.PNPULA_LIK_POISSON), "Poisson"),
    (dict(z_step=1, rho=1e-3), "PSGLA"),
    (dict(z_step=1, rho=1e-3, kappa=1e-3, rho2=1e-3), "second z block"),
    (dict(prior=P.PNPULA_PRIOR_TV, rho=1e-5, kappa=1e-6, z_step=1), "TV"),
    (dict(prior=P.PNPULA_PRIOR_TV), "PSGLA"),
    (dict(prior=P.PNPULA_PRIOR_DDFB), "DDFB"),
    (dict(prior=7), "prior"),
    (dict(halo=3), "halo"),
    (dict(halo=16), "smaller"),
    (dict(sigma=0.0), "sigma"),
    (dict(delta=-1.0), "delta"),
    (dict(rho=-1.0), "rho"),
    (dict(block_y=0), "block"),
    (dict(burn_in=-1), "burn_in"),
])
def test_invalid_configs_are_rejected(over, needle):
    cfg = _cfg(**over)
    with pytest.raises(P.PnpulaError) as e:
        P.Context(cfg)
    assert e.value.code == P.PNPULA_EINVAL
    assert needle in str(e.value)


def test_network_validation():
    wl = W.config(1, ny=32, nx=32, block=32)
    # channels must start and end at 1
    ch, ws, bs = W.denoiser_weights(3, 16, seed=1)
    cfg = P.Config.from_workload(wl)
    cfg2 = P.Config(y=wl.y, kernel=wl.kernel, sigma=wl.sigma, eps=wl.eps, delta=wl.delta,
                    channels=[2, 16, 16, 1], weights=ws, biases=bs)
    for c in (cfg2,):
        with pytest.raises(P.PnpulaError) as e:
            P.Context(c)
        assert e.value.code in (P.PNPULA_EINVAL, P.PNPULA_EDEVICE)
    assert cfg is not None


def test_footprint_is_host_only():
    wl = W.config(2, ny=128, nx=128, block=64)
    b = P.pnpula_footprint(P.Config.from_workload(wl))
    # x ping-pong + y + two 64-channel FP32 activation buffers dominate
    assert b > 2 * 128 * 128 * 64 * 4
    with pytest.raises(P.PnpulaError):
        P.pnpula_footprint(P.Config.from_workload(wl, halo=1))


def test_no_device_is_reported_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(P.PnpulaError) as e:
        P.Context(_cfg())
    assert e.value.code == P.PNPULA_EDEVICE
