"""Benchmark: iterative-thresholding iterations per second (one G + one G^H
per iteration) on a 4096 x 4096 complex64 scene, on one MI355X.

A step is one ITA solve of ``--iters`` iterations (default 100) over the
sparse_4096 workload (1 % log-normal sparse field, 50 % mask, 20 dB),
inputs resident in HBM.  Prints one JSON line with the throughput, the
roofline of the dominant pass kernel (HIP events on the operator's stream)
and the FP64 oracle timed on the host cores.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ITA iterations/s (G+G^H) on 4096² complex64; % HBM peak; batched/grad vs plain"
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per pixel for each pass kind (one read or write of a
# complex64 array = 8 B/pixel; the packed mask = 1/8 B/pixel).
PASS_BYTES = {
    "row_M": 16.0, "row_G": 16.0, "col_fwd": 16.125, "col_inv": 16.0,
    "col_update_threshold": 24.0, "col_residual": 24.125,
}
ITER_BYTES = 80.125  # per pixel per ITA iteration: row G, col R, row M, col A


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_problem(op, shape, seed, density, rate, snr_db, device):
    """Synthetic sparse_4096-style scene on the GPU: y = m o (G x + s n),
    with G the library's operator; lambda from the sparsity rule at X = 0
    (the (k+1)-th largest |M(m o y)|, k = number of nonzeros)."""
    import numpy as np
    import torch

    import inputs
    x = inputs.sparse_field(shape, density, seed)
    k = int(np.count_nonzero(x))
    mask = inputs.random_mask(shape, rate, seed + 1)
    noise = inputs.circular_noise(shape, seed + 2)
    xd = torch.from_numpy(x.astype(np.complex64)).to(device)
    clean = op.apply_G(xd)
    md = torch.from_numpy(mask).to(device)
    p_sig = float((clean.abs() ** 2)[md].mean())
    s = (p_sig / 10.0 ** (snr_db / 10.0)) ** 0.5
    nd = torch.from_numpy(noise.astype(np.complex64)).to(device)
    y = torch.where(md, clean + s * nd, torch.zeros_like(clean))
    b0 = op.apply_GH(y).abs().flatten()
    lam = float(torch.topk(b0, k + 1).values[-1])
    bits = op.pack_mask(md)
    del xd, clean, nd, b0
    return y, bits, lam, k


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def cpu_baseline(shape, seed):
    """The FP64 oracle, as it stands, on the host: one full ITA iteration
    (G, M and the threshold) on the same workload shape."""
    import numpy as np

    import inputs
    from oracle import csa, ita
    threads = len(os.sched_getaffinity(0))
    g = csa.Geometry(inputs.RADAR_STRIPMAP, shape)
    y = inputs.random_complex(shape, seed)
    mask = inputs.random_mask(shape, 0.5, seed + 1)
    y = np.where(mask, y, 0)
    x1, _ = ita.ita(y, mask, 0.5, 1, g)  # builds screens and DFT matrices
    t0 = time.perf_counter()
    ita.ita(y, mask, 0.5, 1, g, x0=x1)  # one iteration with a non-zero iterate
    dt = time.perf_counter() - t0
    return dict(value=1.0 / dt, unit="iterations/s", cores=threads, kind="oracle",
                sample=f"1 ITA iteration (G + G^H + soft threshold, naive FP64 DFTs) on a "
                       f"{shape[0]}x{shape[1]} scene, 50% mask; {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=100, help="ITA iterations per step")
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the event-instrumented region (plain timing only)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the single-scene "
                                   "ITA is not sharded across GPUs (--gpus must be 1)"}))
        sys.exit(2)

    import torch
    import paper_1302_3120_amd as pk
    import inputs

    dev = torch.device("cuda:0")
    shape = (args.size, args.size)
    wl = inputs.workload("sparse_4096")
    op = pk.make_operator(inputs.RADAR_STRIPMAP, shape)
    log(f"bench: building {shape} problem")
    y, bits, lam, k = make_problem(op, shape, wl["seed"], wl["density"], wl["mask_rate"],
                                   wl["snr_db"], dev)
    out = torch.empty_like(y)
    ws = op.workspace(1, dev)
    hist = None

    def step():
        op.ita_solve(y, bits, lam, args.iters, out=out, ws=ws)

    log(f"bench: timing {args.steps} steps x {args.iters} iterations (lambda {lam:.4g}, k {k})")
    dt = time_steps(step, args.steps, args.warmup)
    op.sync_status()
    its = args.steps * args.iters / dt
    n = shape[0] * shape[1]
    rec = {
        "metric": METRIC, "value": its, "unit": "iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"sparse_{shape[0]}: {shape[0]}x{shape[1]} complex64, 1% "
                               f"log-normal sparse field, 50% mask, 20 dB, "
                               f"{args.iters} ITA iterations per step",
                   "shape": list(shape), "iters_per_step": args.iters, "lambda": lam,
                   "nonzeros": k},
        "hbm_frac_algorithmic": ITER_BYTES * n * its / (HBM_PEAK_GBS * 1e9),
    }

    if not args.no_profile:
        # Second timed region with per-launch HIP events on the operator's
        # stream: per-kernel average durations and achieved bandwidth.
        op.profile(True)
        op.profile_read()
        dt2 = time_steps(step, args.steps, 0)
        prof = op.profile_read()
        op.profile(False)
        kernels = {}
        for kind, (ms, cnt) in prof.items():
            avg_us = 1e3 * ms / cnt
            gbytes = PASS_BYTES[kind] * n / 1e9
            kernels[kind] = {"launches": cnt, "avg_us": avg_us, "algo_GB": gbytes,
                             "GBs": gbytes / (avg_us * 1e-6), "total_ms": ms}
        dom = max(kernels, key=lambda kk: kernels[kk]["total_ms"])
        kd = kernels[dom]
        rec["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": kd["GBs"],
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": kd["GBs"] / HBM_PEAK_GBS, "traffic": None}
        rec["kernels"] = kernels
        rec["profiled_region_iterations_per_s"] = args.steps * args.iters / dt2

    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on the host (one iteration)")
        rec["cpu_baseline"] = cpu_baseline(shape, 1234)

    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
