"""Throughput of the PnP-ULA hot path on one MI355X.

One step = one full iteration x^(t) -> x^(t+1) of the sampler over the whole
image (denoiser layers, fused likelihood gradient / z draw / update /
statistics).  Default workload: 4096 x 4096 image, 9x9 Gaussian blur,
sigma = 0.02, 8 x 8 blocks of 512 x 512 with an 8-pixel halo, 8-layer
64-channel denoiser in bf16 with FP32 accumulation, split rho = sigma^2,
synthetic seeded inputs.  Timed steps run after burn-in, so the Welford
statistics (and their FP64 merges) are part of every step.

Prints one JSON line.  Extra fields: the same workload in FP32 and e4m3 for
comparison, the roofline of the dominant kernel (middle convolution layers,
matrix-core bound) and of the fused update kernel (HBM bound), and the FP64
oracle timed on the host over a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {0: 157.3, 1: 2500.0, 2: 5000.0}     # MI355X dense: fp32, bf16, fp8
PEAK_HBM_GBS = 8000.0
DTYPE = {0: "fp32", 1: "bf16", 2: "fp8_e4m3"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--precision", type=int, default=None)
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-region", type=int, default=2048)
    ap.add_argument("--serving", action="store_true",
                    help="continuous-batching run: Poisson job arrivals, p50/p99 latency")
    ap.add_argument("--jobs", type=int, default=64)
    ap.add_argument("--iters-scale", type=float, default=0.1,
                    help="serving: fraction of the 1000-5000 iterations each job runs")
    ap.add_argument("--no-serving-leg", action="store_true",
                    help="skip the bounded serving pass of the default run")
    ap.add_argument("--leg-jobs", type=int, default=32)
    ap.add_argument("--leg-iters-scale", type=float, default=0.05)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--no-next", action="store_true",
                    help="skip the pass over the paper's other data terms and priors")
    ap.add_argument("--next-steps", type=int, default=5)
    ap.add_argument("--only-next", default=None,
                    help="run only this row of the pass (poisson, tv, ddfb, blur65, blur129)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (three times): the "
                         "reference for scaling the FETCH_SIZE / WRITE_SIZE counters")
    return ap.parse_args()


PROFILE_MD = os.path.join(ROOT, "profiles", "denoiser_step_4096sq_bf16.md")
# matrix-core kernel classes of the library's profiler: (kernel, row of the
# rocprofv3 summary, middle layers per launch, extra flops per pixel)
MFMA_CLASSES = {
    0: ("conv_mid_kernel", "conv_mid_rr_kernel<false, false>", 1, 0),
    4: ("conv_mid_rr_kernel<true,false> (first layer fused)", "conv_mid_rr_kernel<true, false>",
        1, 2 * 9 * 64),
    5: ("conv_mid_rr_kernel<false,true> (last layer partials fused)",
        "conv_mid_rr_kernel<false, true>", 1, 2 * 9 * 64),
    6: ("conv_pair_ws_kernel (two bf16 middle layers, one per wave group)", "conv_pair_ws_kernel",
        2, 0),
}
# class 6 for e4m3 networks
PAIR8_CLASS = ("e4m3 layer pairs (conv_pair8_ws_kernel; conv_pair8_kernel with the first or last "
               "layer), averaged over the step's pair launches", "conv_pair8", 2, 0)


# sources of the kernels the bf16 step runs (the denoiser layers and the
# fused update) and the layout they share: the committed summary's figures
# hold while these are unchanged
STEP_SOURCES = ("conv.hip", "device_common.h", "kernels.h", "update.hip")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2511_00870_amd", "csrc")
    for name in sorted(STEP_SOURCES):
        h.update(name.encode())
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_avg_ms(row):
    """Average launch duration (ms) of the kernel named `row` in the committed
    rocprofv3 kernel-trace summary, or None when the kernel sources changed
    since it was taken."""
    try:
        with open(PROFILE_MD) as fh:
            text = fh.read()
    except OSError:
        return None
    import re
    m = re.search(r"`([0-9a-f]{64})`", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    for line in text.splitlines():
        if f"pnp::{row}(" in line and line.count("|") == 7:
            cells = [c.strip() for c in line.strip("|").split("|")]
            return float(cells[2]) / 1e3
    return None


def recorded_traffic(row):
    """HBM bytes per launch of the kernel named `row` from the committed
    FETCH_SIZE / WRITE_SIZE summary (already scaled by the plain-copy factor),
    or None when the kernel sources changed since those counters were taken."""
    import re
    try:
        with open(PROFILE_MD) as fh:
            text = fh.read()
    except OSError:
        return None
    m = re.search(r"`([0-9a-f]{64})`", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    for line in text.splitlines():
        if f"pnp::{row}(" in line and line.count("|") == 6:
            cells = [c.strip() for c in line.strip("|").split("|")]
            return (float(cells[3]) + float(cells[4])) * 1e9
    return None


def fp8_scales(ctx_fp32, wl, x):
    """Power-of-two e4m3 activation scales from the library's own FP32
    calibration pass (twice the largest |input| of each layer)."""
    from paper_2511_00870_amd import workloads as W
    amax = ctx_fp32.calibrate(x)
    fmt = W.layer_formats(wl.n_layers, 2)
    return [float(2.0 ** np.ceil(np.log2(2 * a / 448))) if f == 2 else 1.0
            for a, f in zip(amax, fmt)]


def run_gpu(wl, precision, steps, warmup, stream, act_scales=None, profile=True,
            classes=range(7)):
    import torch
    from paper_2511_00870_amd import pnpula as P
    cfg = P.Config.from_workload(wl, precision=precision, act_scales=act_scales, stream=stream)
    ctx = P.Context(cfg)
    # start after burn-in so every timed step updates the statistics
    x0 = np.clip(wl.xbar, 0, 1).astype(np.float32)
    ctx.set_state(x0, wl.burn_in + 1)
    ctx.step(warmup)
    torch.cuda.synchronize()
    if profile:
        ctx.profile(True)
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rc = ctx.sync()
    prof = {c: ctx.profile_read(c) for c in classes} if profile else None
    ctx.close()
    return dt, rc, prof


# kernels of the other data terms and priors, per profiler class: class 7
# is the prior other than the CNN (TV coupling term or the DDFB stages),
# class 8 the z-steps, class 9 the large-blur correlation passes, class 3
# the update
def next_workloads(rows=None):
    """The paper's other data terms and priors at 4096^2 (Sec. III-A2, III-A3,
    III-B, II-B1 Example 3), each with its own dominant kernel."""
    from paper_2511_00870_amd import workloads as W
    n = 4096
    out = {}
    want = (lambda k: rows is None or k == rows)
    if want("poisson"):
        out["poisson"] = W.poisson_workload("4096x4096 Poisson deconvolution (eta 250, PSGLA z1 KL "
                                            "+ z2 on R+), blur 9, 8x64 bf16 CNN", n, n,
                                            W.gaussian_kernel(9, 2.0), 512, 8, 8, 64, 1, 2000,
                                            200, 6000)
    if want("tv"):
        out["tv"] = W.tv_workload("4096x4096 TV prior (AXDA-PSGLA, beta 40), blur 9", n, n,
                                  W.gaussian_kernel(9, 2.0), 0.02, 512, 8, 2000, 200, 7000)
    if want("ddfb"):
        out["ddfb"] = W.ddfb_workload("4096x4096 DDFB denoiser K=4 F=64, blur 9", n, n, 9, 2.0,
                                      0.02, 512, 8, 2000, 200, 8000, n_layers=4, features=64)
    for L in (65, 129):
        key = f"blur{L}"
        if not want(key):
            continue
        wl = W.make_workload(f"4096x4096 motion blur {L}x{L} (non-separable), 8x64 bf16 CNN",
                             n, n, L=5, sigma_k=1.0, sigma=0.02, block=n, halo=L - 1,
                             n_layers=8, features=64, precision=1, iters=2000, burn_in=200,
                             seed=9000 + L)
        k = W.motion_blur_kernel(L, seed=L)
        wl.kernel = k
        wl.y = W.observe(wl.xbar, k, wl.sigma, None, 9001 + L)
        out[key] = wl
    return out


def next_rows(a, stream):
    """Throughput of each of the other rows at 4096^2 and the roofline of
    the kernel class that row adds: HBM for the TV and z-step kernels (their
    algorithmic bytes per pixel), vector ALU for the DDFB stages and the
    large-blur correlations (their algorithmic flops per pixel)."""
    res = {}
    for key, wl in next_workloads(a.only_next).items():
        npx = wl.ny * wl.nx
        try:
            dt, rc, prof = run_gpu(wl, wl.precision, a.next_steps, 1, stream, None,
                                   classes=range(10))
        except Exception as e:  # report, do not hide
            res[key] = {"error": str(e)}
            continue
        r = {"workload": wl.name, "value": round(npx * a.next_steps / dt / 1e6, 2),
             "unit": "Mpixel*iter/s", "ms_per_step": round(dt / a.next_steps * 1e3, 4),
             "status": rc,
             "kernel_ms_per_step": {n: round(prof[c][0] / a.next_steps, 4) for c, n in
                                    [(3, "update"), (6, "conv_pair"), (4, "conv_first_mid"),
                                     (5, "conv_mid_last"), (2, "conv_last"),
                                     (7, "prior"), (8, "z_step"), (9, "blur_passes")]
                                    if prof[c][1]}}
        def avg(c):
            return prof[c][0] / prof[c][1] / 1e3
        if key == "tv":
            # prior term: x read 4 + zh, zv read 8 + G write 4; z-step: x 4 + z r/w 16
            r["roofline"] = {"bound": "hbm", "kernel": "tv_prior_kernel",
                             "achieved": round(16 * npx / avg(7) / 1e9, 1), "peak": PEAK_HBM_GBS,
                             "unit": "GB/s", "frac": round(16 * npx / avg(7) / 1e9 / PEAK_HBM_GBS, 4),
                             "avg_launch_ms": round(avg(7) * 1e3, 4), "bytes_per_launch": 16 * npx}
            r["roofline_z_step"] = {"bound": "hbm", "kernel": "zstep_tv_kernel",
                                    "achieved": round(20 * npx / avg(8) / 1e9, 1),
                                    "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                    "frac": round(20 * npx / avg(8) / 1e9 / PEAK_HBM_GBS, 4),
                                    "avg_launch_ms": round(avg(8) * 1e3, 4),
                                    "bytes_per_launch": 20 * npx}
        elif key == "poisson":
            # z-step: x 4 + y 4 + z1, z2 read + write 16
            r["roofline"] = {"bound": "hbm", "kernel": "zstep_psgla_kernel",
                             "achieved": round(24 * npx / avg(8) / 1e9, 1), "peak": PEAK_HBM_GBS,
                             "unit": "GB/s", "frac": round(24 * npx / avg(8) / 1e9 / PEAK_HBM_GBS, 4),
                             "avg_launch_ms": round(avg(8) * 1e3, 4), "bytes_per_launch": 24 * npx}
        elif key == "ddfb":
            K, F = len(wl.ddfb_gamma), wl.ddfb_weights.shape[1]
            fl = 2.0 * 2 * K * 9 * F * npx        # K forward + K adjoint convolutions
            per_iter = prof[7][0] / a.next_steps / 1e3
            r["roofline"] = {"bound": "mfma", "kernel": "ddfb_stage_kernel (all K stages, FP32 matrix cores)",
                             "achieved": round(fl / per_iter / 1e12, 2), "peak": 157.3,
                             "unit": "TFLOP/s", "frac": round(fl / per_iter / 1e12 / 157.3, 4),
                             "ms_per_iteration": round(per_iter * 1e3, 4),
                             "flops_per_iteration": fl}
        else:
            L = wl.kernel.shape[0]
            fl = 2.0 * L * L * npx                # one correlation pass
            r["roofline"] = {"bound": "mfma", "kernel": f"blur_big_kernel ({L}x{L}, FP32 matrix cores)",
                             "achieved": round(fl / avg(9) / 1e12, 2), "peak": 157.3,
                             "unit": "TFLOP/s", "frac": round(fl / avg(9) / 1e12 / 157.3, 4),
                             "avg_launch_ms": round(avg(9) * 1e3, 4), "flops_per_launch": fl}
        res[key] = r
    return res


def cpu_baseline(wl, region):
    import oracle.oracle as O
    oc = O.Chain.from_workload(wl, block=0)
    x = np.clip(wl.xbar, 0, 1)
    y0, x0 = wl.ny // 2 - region // 2, wl.nx // 2 - region // 2
    t0 = time.perf_counter()
    oc.step_region(x, wl.burn_in + 1, y0, x0, region, region)
    dt = time.perf_counter() - t0
    return {"value": round(region * region / dt / 1e6, 6), "unit": "Mpixel*iter/s",
            "cores": O.num_threads(), "kind": "oracle",
            "sample": f"one FP64 iteration of a {region}x{region} region (plus its "
                      f"max(2r,K) halo) of the same workload, {dt:.1f} s"}


def serving(a, stream, n_jobs=None, iters_scale=None):
    """Jobs arrive by a Poisson process (20/s); each is submitted at its
    arrival, the server ticks continuously, latency = completion - arrival."""
    from paper_2511_00870_amd import pnpula as P
    from paper_2511_00870_amd import workloads as W
    n_jobs = a.jobs if n_jobs is None else n_jobs
    iters_scale = a.iters_scale if iters_scale is None else iters_scale
    lo, hi = max(1, int(1000 * iters_scale)), max(1, int(5000 * iters_scale))
    jobs = W.serving_jobs(n_jobs=n_jobs, iters=(lo, hi))
    net = jobs[0].workload
    srv = P.Server(net.channels, net.weights, net.biases, precision=P.PNPULA_BF16,
                   max_slots=a.slots, stream=stream)
    cfgs = [P.Config.from_workload(j.workload) for j in jobs]
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    submitted, done, lat = {}, set(), []
    nxt = 0
    work = 0.0
    while len(done) < len(jobs):
        now = time.perf_counter() - t0
        while nxt < len(jobs) and jobs[nxt].arrival_s <= now:
            jid = srv.submit(cfgs[nxt], jobs[nxt].workload.iters)
            submitted[jid] = nxt
            nxt += 1
        if len(submitted) == len(done):
            time.sleep(max(0.0, jobs[nxt].arrival_s - now))
            continue
        srv.tick()
        now = time.perf_counter() - t0
        for jid, k in submitted.items():
            if k in done or not srv.poll(jid):
                continue
            m, v, n = srv.result(jid)
            done.add(k)
            wl = jobs[k].workload
            lat.append(now - jobs[k].arrival_s)
            work += wl.ny * wl.nx * wl.iters
    span = time.perf_counter() - t0
    lat = np.array(lat)
    return {
        "metric": "p50/p99 job latency and aggregate Mpixel*Langevin-iter/s (serving)",
        "value": round(work / span / 1e6, 2), "unit": "Mpixel*iter/s", "n_gpus": 1,
        "p50_latency_s": round(float(np.percentile(lat, 50)), 3),
        "p99_latency_s": round(float(np.percentile(lat, 99)), 3),
        "makespan_s": round(span, 2), "higher_is_better": True, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"serving: {n_jobs} jobs, Poisson 20/s, sides 256-2048, "
                               f"blur 5-9 (+50% mask), iterations {lo}-{hi}, 8x64 bf16 "
                               f"denoiser, {a.slots} slots"},
    }


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the sampler runs on one GPU per process; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2511_00870_amd import workloads as W
    from paper_2511_00870_amd.accounting import fused_update_bytes_per_pixel
    torch.cuda.set_device(0)
    if a.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4, "copies": 3}), flush=True)
        return
    stream = torch.cuda.current_stream().cuda_stream
    if a.serving:
        print(json.dumps(serving(a, stream)), flush=True)
        return
    if a.only_next:
        print(json.dumps(next_rows(a, stream)), flush=True)
        return
    wl = W.config(a.config)
    prec = wl.precision if a.precision is None else a.precision
    npx = wl.ny * wl.nx
    F = wl.channels[1]
    scales = None
    if prec == 2:
        from paper_2511_00870_amd import pnpula as P
        c32 = P.Context(P.Config.from_workload(wl, precision=0, stream=stream))
        scales = fp8_scales(c32, wl, np.clip(wl.xbar, 0, 1).astype(np.float32))
        c32.close()
    dt, rc, prof = run_gpu(wl, prec, a.steps, a.warmup, stream, scales)
    ms = dt / a.steps * 1e3
    value = npx * a.steps / dt / 1e6
    upd_ms, upd_n = prof[3]
    # the dominant matrix-core kernel: the class with the largest total time
    busy = [c for c in MFMA_CLASSES if prof[c][1]]
    out = {
        "metric": "Mpixel*Langevin-iter/s at 4096^2 (BF16/FP8 vs FP32); p50/p99 job latency",
        "value": round(value, 2), "unit": "Mpixel*iter/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[prec], "data": "synthetic",
        "config": {"workload": wl.name, "image": [wl.ny, wl.nx], "blur": int(wl.kernel.shape[0]),
                   "blocks": [wl.block_y, wl.block_x], "halo": wl.halo,
                   "denoiser": f"{wl.n_layers}x{F}", "split_rho": wl.rho, "iters": wl.iters,
                   "burn_in": wl.burn_in},
        "status": rc,
    }
    if busy:
        c = max(busy, key=lambda k: prof[k][0])
        name, row, layers, extra = PAIR8_CLASS if (c == 6 and prec == 2) else MFMA_CLASSES[c]
        avg = prof[c][0] / prof[c][1] / 1e3
        flops_launch = (layers * 2.0 * 9 * F * F + extra) * npx
        ach = flops_launch / avg / 1e12
        # counters exist for the default bf16 workload only
        traffic = recorded_traffic(row) if (a.config == 3 and prec == 1) else None
        if traffic is not None:
            traffic = round(traffic)
        out["roofline"] = {"bound": "mfma", "kernel": name,
                           "achieved": round(ach, 2), "peak": PEAK_TFLOPS[prec],
                           "unit": "TFLOP/s", "frac": round(ach / PEAK_TFLOPS[prec], 4),
                           "traffic": traffic, "avg_launch_ms": round(avg * 1e3, 4),
                           "flops_per_launch": flops_launch}
        # the same kernel's average in the committed rocprofv3 summary, and the
        # fraction it gives (present while the kernel sources are unchanged)
        pavg = recorded_avg_ms(row) if (a.config == 3 and prec == 1) else None
        if pavg is not None:
            out["roofline"]["profile_avg_launch_ms"] = round(pavg, 4)
            out["roofline"]["profile_frac"] = round(
                flops_launch / (pavg / 1e3) / 1e12 / PEAK_TFLOPS[prec], 4)
    if upd_n:
        avg = upd_ms / upd_n / 1e3
        byt = fused_update_bytes_per_pixel(True, wl.mask is not None, wl.welford_window) * npx
        out["roofline_fused_update"] = {"bound": "hbm", "achieved": round(byt / avg / 1e9, 1),
                                        "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                        "frac": round(byt / avg / 1e9 / PEAK_HBM_GBS, 4),
                                        "avg_launch_ms": round(avg * 1e3, 4),
                                        "bytes_per_launch": byt}
    out["kernel_ms_per_step"] = {name: round(prof[c][0] / a.steps, 4) for c, name in
                                 [(0, "conv_mid"), (1, "conv_first"), (2, "conv_last"),
                                  (3, "fused_update"), (4, "conv_first_mid"),
                                  (5, "conv_mid_last"), (6, "conv_pair")]}
    if not a.no_compare:
        comp = {}
        for p in (0, 1, 2):
            if p == prec:
                comp[DTYPE[p]] = round(value, 2)
                continue
            try:
                sc = None
                if p == 2:
                    from paper_2511_00870_amd import pnpula as P
                    c32 = P.Context(P.Config.from_workload(wl, precision=0, stream=stream))
                    sc = fp8_scales(c32, wl, np.clip(wl.xbar, 0, 1).astype(np.float32))
                    c32.close()
                n = 4 if p == 0 else a.steps
                d, _, _ = run_gpu(wl, p, n, 1, stream, sc, profile=False)
                comp[DTYPE[p]] = round(npx * n / d / 1e6, 2)
            except Exception as e:  # report, do not hide
                comp[DTYPE[p]] = f"error: {e}"
        out["compare_precisions"] = comp
    if not a.no_serving_leg:
        # a bounded continuous-batching pass: latency percentiles and the
        # aggregate rate of a Poisson job stream (fewer, shorter jobs than the
        # full 256-job serving workload, which bench.py --serving runs)
        sv = serving(a, stream, a.leg_jobs, a.leg_iters_scale)
        out["p50_latency_s"] = sv["p50_latency_s"]
        out["p99_latency_s"] = sv["p99_latency_s"]
        out["serving"] = {k: sv[k] for k in ("value", "unit", "p50_latency_s", "p99_latency_s",
                                             "makespan_s")}
        out["serving"]["workload"] = sv["config"]["workload"]
    if not a.no_next:
        out["next_rows"] = next_rows(a, stream)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, a.cpu_region)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
