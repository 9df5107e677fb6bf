"""pnpula_data_grad_noalloc (the entry point for callers that cannot
allocate device memory) against pnpula_data_grad on the same inputs, two
calls in a row, the second on a smaller image: both calls share the static
residual buffer, and each must equal the allocating entry point bitwise (the
same kernels run on the same values) and the oracle within the FP32 bar."""
import numpy as np
import pytest

import oracle.oracle as O
from paper_2511_00870_amd import pnpula as P
from paper_2511_00870_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ctx(ny, nx, L, mask_p, seed):
    wl = W.make_workload("g", ny, nx, L=5, sigma_k=1.0, sigma=0.02, block=max(ny, nx),
                         halo=max(L - 1, 4), n_layers=4, features=16, precision=0, iters=1,
                         burn_in=0, seed=seed, mask_p=mask_p, split=False)
    k = W.motion_blur_kernel(L, seed=L)
    wl.kernel = k
    wl.y = W.observe(wl.xbar, k, wl.sigma, wl.mask, seed + 1)
    return wl, P.Context(P.Config.from_workload(wl))


def test_noalloc_data_grad_matches_allocating_entry_point():
    import torch
    dev = torch.device("cuda:0")
    for (ny, nx, L, mask_p) in [(300, 280, 65, 0.5), (90, 70, 9, None)]:
        print(f"case noalloc data gradient {ny}x{nx} L={L} mask={mask_p}", flush=True)
        wl, ctx = _ctx(ny, nx, L, mask_p, 31 + L)
        x = np.random.default_rng(L).random((ny, nx)).astype(np.float32)
        ref = ctx.data_grad(x)
        tx = torch.from_numpy(x).to(dev)
        tg = torch.full((ny, nx), float("nan"), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        ctx.data_grad_noalloc(tx, tg)
        assert ctx.sync() == P.PNPULA_OK
        g = tg.cpu().numpy()
        assert np.array_equal(g, ref)
        oref = O.Chain.from_workload(wl, block=0).data_grad(x.astype(np.float64), 0)
        e = float(np.linalg.norm(g - oref) / np.linalg.norm(oref))
        print(f"  bitwise equal to pnpula_data_grad; rel to the oracle {e:.2e}", flush=True)
        assert e <= 1e-5


def test_noalloc_rejects_images_beyond_the_static_buffer():
    import torch
    ny, nx = 2900, 2900                      # 8.41 M pixels > 2^23
    wl = W.make_workload("g", ny, nx, L=5, sigma_k=1.0, sigma=0.02, block=ny, halo=4,
                         n_layers=4, features=16, precision=0, iters=1, burn_in=0, seed=3,
                         split=False)
    ctx = P.Context(P.Config.from_workload(wl))
    t = torch.zeros((ny, nx), dtype=torch.float32, device="cuda:0")
    with pytest.raises(P.PnpulaError) as e:
        ctx.data_grad_noalloc(t, t)
    assert e.value.code == P.PNPULA_EINVAL
