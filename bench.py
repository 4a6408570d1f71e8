"""Benchmark: iterative-thresholding iterations per second (one G + one G^H
per iteration) on a 4096 x 4096 complex64 scene, on one MI355X.

A step is one ITA solve of ``--iters`` iterations (default 100) over the
sparse_4096 workload (1 % log-normal sparse field, 50 % mask, 20 dB),
inputs resident in HBM.  Prints one JSON line with the throughput, the
roofline of the dominant pass kernel (HIP events on the operator's stream)
and the FP64 oracle timed on the host cores.
"""

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ITA iterations/s (G+G^H) on 4096² complex64; % HBM peak; batched/grad vs plain"
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per pixel for each pass kind (one read or write of a
# complex64 array = 8 B/pixel; the packed mask = 1/8 B/pixel, read once at
# t = 0, where the copy of m o y with unsampled entries marked is written).
PASS_BYTES = {
    "row_M": 16.0, "row_G": 16.0, "col_fwd": 24.125, "col_inv": 16.0,
    "col_update_threshold": 24.0, "col_residual": 24.0,
}
# Per pixel per ITA iteration (row G, col R, row M, col A: 80 B) plus the
# mask (1/8 B): the conventional figure for the fraction of HBM peak.
ITER_BYTES = 80.125


def sparse_update_bytes(nnz_frac):
    """Algorithmic bytes per pixel of the sparse-iterate update pass: Z read
    and F_eta X+ written (16), and the iterate's nonzeros read and written,
    each as an 8-byte value and a 4-byte position (2 x 12 x the nonzero
    fraction).  The pass's own format (a wave mask, 32-byte records of the
    threads with nonzeros) moves somewhat more; that overhead is not
    counted."""
    return 16.0 + 24.0 * nnz_frac
# Kernel symbol of each pass kind; {v} is the plan variant (the residual
# column pass at 4096 runs variant 1, see column_variant in cssar_api.hip).
KIND_SYMBOL = {
    "row_M": "row_pass_kernel<cssar::Plan<{n}, {v}>, 0>",
    "row_G": "row_pass_kernel<cssar::Plan<{n}, {v}>, 1>",
    "col_fwd": "col_pass_kernel<cssar::Plan<{n}, {v}>, 0>",
    "col_inv": "col_pass_kernel<cssar::Plan<{n}, {v}>, 1>",
    "col_update_threshold": "col_pass_kernel<cssar::Plan<{n}, {v}>, 2>",
    "col_residual": "col_pass_kernel<cssar::Plan<{n}, {v}>, 3>",
    "col_update_sparse": "col_pass_kernel<cssar::Plan<{n}, {v}>, 11>",
}
# plan variant of a pass kind at a line length, where it is not 0 (the
# library's column_variant and row_variant)
KIND_VARIANT = {("col_residual", 4096): 1, ("col_update_threshold", 4096): 2,
                ("col_update_sparse", 4096): 2, ("col_update_threshold", 2048): 1,
                ("col_update_sparse", 2048): 1, ("col_residual", 2048): 1, ("row_M", 8192): 1,
                ("row_G", 8192): 1,
                ("col_fwd", 8192): 1, ("col_inv", 8192): 1}


def kind_symbol(kind, n):
    """Kernel symbol of a pass kind at line length n."""
    return KIND_SYMBOL[kind].format(n=n, v=KIND_VARIANT.get((kind, n), 0))
# Counter-based HBM bytes per dispatch, written by --rocprof-summary from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) and a copy-kernel calibration.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ita_passes_sparse_4096.md")
CAL_MIB = 256  # size of the calibration copy (read and written once each)


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


def make_batched_problem(ops, wl, device):
    """The 64-scene workload on the GPU (torch's seeded generator): per scene
    a sparse scene of 50-300 point targets, y = m o (G x + s n) with the
    library's G at 20 dB, mask rate U(0.3, 0.7), lambda by the sparsity rule."""
    import numpy as np
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(wl["seed"])
    r = np.random.default_rng(wl["seed"])
    ys, bits, lams = [], [], []
    for op in ops:
        na, nr = op.shape
        k = int(r.integers(wl["targets"][0], wl["targets"][1] + 1))
        rate = float(r.uniform(*wl["mask_rate"]))
        x = torch.zeros(na * nr, dtype=torch.complex64, device=device)
        idx = torch.randperm(na * nr, generator=g, device=device)[:k]
        amp = 0.5 + 0.5 * torch.rand(k, generator=g, device=device)
        ph = 2 * np.pi * torch.rand(k, generator=g, device=device)
        x[idx] = torch.polar(amp, ph)
        clean = op.apply_G(x.view(na, nr))
        m = torch.rand(na, nr, generator=g, device=device) < rate
        p_sig = float((clean.abs() ** 2)[m].mean())
        sn = (p_sig / 10.0 ** (wl["snr_db"] / 10.0)) ** 0.5
        n = torch.randn(na, nr, dtype=torch.complex64, generator=g, device=device)
        y = torch.where(m, clean + sn * n, torch.zeros_like(clean))
        lams.append(float(torch.topk(op.apply_GH(y).abs().flatten(), k + 1).values[-1]))
        ys.append(y)
        bits.append(op.pack_mask(m))
    return ys, bits, lams


def bench_batched(steps, iters, device):
    """Batched solver on the 64-scene workload against the plain loop of
    per-scene solves, same GPU, same inputs."""
    import torch
    import inputs
    import paper_1302_3120_amd as pk
    wl = inputs.workload("batched_64")
    shapes = inputs.batched_shapes(wl["count"], wl["seed"], wl["sizes"])
    ops = [pk.make_operator(inputs.RADAR_STRIPMAP, sh) for sh in shapes]
    log(f"bench: batched workload, {len(shapes)} scenes")
    ys, bits, lams = make_batched_problem(ops, wl, device)
    px = sum(a * b for a, b in shapes)
    outs = [torch.empty_like(y) for y in ys]
    wss = [op.workspace(1, device) for op in ops]

    def plain():
        for s, op in enumerate(ops):
            op.ita_solve(ys[s], bits[s], lams[s], iters, out=outs[s], ws=wss[s])

    t_plain = time_steps(plain, steps, 1)
    del wss
    b = pk.make_batch(ops)
    ws = b.workspace(device)
    t0 = time.perf_counter()
    b.autotune(ws)
    t_tune = time.perf_counter() - t0
    bouts = [torch.empty_like(y) for y in ys]

    def batched():
        b.ita_solve(ys, bits, lams, iters, outs=bouts, ws=ws)

    t_batch = time_steps(batched, steps, 1)
    # the launch mode the autotuner did not pick, measured too (graph replay
    # of the middle iterations, or direct launches)
    tuned_graph = "graph=1" in b.describe()
    b.set_graph(not tuned_graph)
    t_other = time_steps(batched, steps, 1)
    b.set_graph(tuned_graph)
    t_graph, t_direct = (t_batch, t_other) if tuned_graph else (t_other, t_batch)
    b.sync_status()
    worst = 0.0
    for o, r in zip(bouts, outs):
        worst = max(worst, float((o - r).abs().pow(2).sum().sqrt() / r.abs().pow(2).sum().sqrt()))
    its_b = steps * iters / t_batch
    its_p = steps * iters / t_plain
    return {
        "workload": f"batched_64: {len(shapes)} scenes, dims from {list(wl['sizes'])}, "
                    f"{px / 1e6:.1f} Mpx, {iters} iterations per step",
        "iterations_per_s": its_b, "plain_loop_iterations_per_s": its_p,
        "speedup_vs_plain_loop": its_b / its_p,
        "graph_replay_iterations_per_s": steps * iters / t_graph,
        "direct_launch_iterations_per_s": steps * iters / t_direct,
        "tuned_launch_mode": "graph" if tuned_graph else "direct",
        "Mpx_iterations_per_s": its_b * px / 1e6,
        "algorithmic_GBs": its_b * px * ITER_BYTES / 1e9,
        "hbm_frac_algorithmic": its_b * px * ITER_BYTES / (HBM_PEAK_GBS * 1e9),
        "rel_l2_vs_plain_loop": worst, "autotune_s": t_tune,
        "choices": b.describe().strip().splitlines(),
    }


def bench_grad(steps, device):
    """Differentiated workload (1024 x 1024, 100 point targets, 50 % mask,
    20 dB, K = 20, checkpoint every 5; raw data through the library's G):
    forward with checkpoints + reverse pass for L = ||X^(K) - x*||^2,
    against the plain K-iteration solve on the same inputs, and the
    gradient's error against the FP64 oracle's, stored for the same recipe
    (tests/golden/grad_1024.npz, written by tests/golden/grad_1024.py)."""
    import numpy as np
    import torch
    import inputs
    import paper_1302_3120_amd as pk
    wl, xt, mask, noise, pick = inputs.gradient_problem_parts("grad_1024", 256)
    shape, K, every = wl["shape"], wl["iters"], wl["every"]
    op = pk.make_operator(inputs.RADAR_STRIPMAP, shape)
    md = torch.from_numpy(mask).to(device)
    xtd = torch.from_numpy(xt.astype(np.complex64)).to(device)
    clean = op.apply_G(xtd)
    s = float((clean.abs() ** 2)[md].mean() / 10.0 ** (wl["snr_db"] / 10.0)) ** 0.5
    nd = torch.from_numpy(noise.astype(np.complex64)).to(device)
    y = torch.where(md, clean + s * nd, torch.zeros_like(clean))
    bits = op.pack_mask(md)
    lam = float(torch.topk(op.apply_GH(y).abs().flatten(), wl["targets"] + 1).values[-1])
    out = torch.empty_like(y)
    ws = op.workspace(1, device)

    def plain():
        op.ita_solve(y, bits, lam, K, out=out, ws=ws)

    def fwd_bwd():
        xk, ck = op.ita_forward(y, bits, lam, K, every)
        op.ita_backward(y, bits, lam, K, every, ck, 2.0 * (xk - xtd))

    t_plain = time_steps(plain, steps, 1)
    t_grad = time_steps(fwd_bwd, steps, 1)
    rec = {
        "workload": f"grad_1024: {shape[0]}x{shape[1]}, 100 point targets, 50% mask, 20 dB, "
                    f"K = {K} unrolled iterations, checkpoint every {every}; gradients of "
                    f"||X(K) - x*||^2 in y, lambda, K_a, K_r",
        "forward_backward_ms": 1e3 * t_grad / steps, "plain_solve_ms": 1e3 * t_plain / steps,
        "cost_vs_plain_solve": t_grad / t_plain,
        "iterations_per_s_forward_backward": steps * K / t_grad,
    }
    gold_path = os.path.join(ROOT, "tests", "golden", "grad_1024.npz")
    if os.path.exists(gold_path):
        gold = np.load(gold_path, allow_pickle=False)
        yd = y.clone().requires_grad_(True)
        lt = torch.tensor(lam, dtype=torch.float64, requires_grad=True)
        ka = torch.tensor(pk.ka_of(inputs.RADAR_STRIPMAP), dtype=torch.float64, requires_grad=True)
        kr = torch.tensor(float(inputs.RADAR_STRIPMAP["Kr"]), dtype=torch.float64, requires_grad=True)
        x = pk.ITAUnrolled.apply(yd, lt, ka, kr, md, K, every, inputs.RADAR_STRIPMAP)
        loss = (x - xtd).abs().pow(2).sum()
        loss.backward()
        yb = yd.grad.flatten()[torch.from_numpy(gold["pick"]).to(device)].cpu().numpy()
        want = gold["ybar"]
        err = {
            "lambda": abs(float(lt.grad) - float(gold["lbar"])) / abs(float(gold["lbar"])),
            "K_a": abs(float(ka.grad) - float(gold["kabar"])) / abs(float(gold["kabar"])),
            "K_r": abs(float(kr.grad) - float(gold["krbar"])) / abs(float(gold["krbar"])),
            "y_sampled": float(np.linalg.norm(yb - want) / np.linalg.norm(want)),
            "loss": abs(float(loss.detach()) - float(gold["loss"])) / float(gold["loss"]),
        }
        rec["rel_err_vs_oracle"] = err
        rec["max_rel_err_vs_oracle"] = max(err.values())
        rec["lambda_rel_diff_vs_oracle"] = abs(lam - float(gold["lam"])) / float(gold["lam"])
    return rec


def bench_adaptive(op, y, bits, k, iters, steps, device):
    """The iteration with the adaptive step and threshold of Section IV.B
    (cssar_ita_solve_adaptive, sparsity k) on the headline scene: iterations/s
    and the average duration of each pass kind from per-launch HIP events."""
    import torch
    out = torch.empty_like(y)
    ws = op.workspace(2, device)

    def step():
        op.ita_solve_adaptive(y, bits, k, iters, out=out, ws=ws)

    t = time_steps(step, steps, 1)
    op.profile(True)
    op.profile_read()
    step()
    prof = op.profile_read()
    op.profile(False)
    _, mu, lam, _ = op.ita_solve_adaptive(y, bits, k, iters, out=out, ws=ws)
    return {
        "workload": f"the same scene, k = {k} (its nonzero count), {iters} iterations per step",
        "iterations_per_s": steps * iters / t,
        "passes_avg_us": {kind: 1e3 * ms / cnt for kind, (ms, cnt) in prof.items()},
        "passes_launches": {kind: cnt for kind, (ms, cnt) in prof.items()},
        "mu_last": float(mu[-1]), "lambda_last": float(lam[-1]),
    }


def bench_safeguarded(op, y, bits, k, iters, steps, device, c=0.01, kappa=2.0, max_shrinks=2):
    """The adaptive iteration with the support-change safeguard of its step
    (cssar_ita_solve_safeguarded: after a support change, the bound
    (1 - c) ||X+ - X||^2 / ||m o G(X+ - X)||^2 and up to max_shrinks shrinks of
    the step per iteration) on the headline scene: iterations/s, the shrinks
    taken and the average duration of each pass kind."""
    import torch
    out = torch.empty_like(y)
    ws = op.workspace(3, device)

    def step():
        op.ita_solve_safeguarded(y, bits, k, iters, c=c, kappa=kappa, max_shrinks=max_shrinks,
                                 out=out, ws=ws)

    t = time_steps(step, steps, 1)
    op.profile(True)
    op.profile_read()
    step()
    prof = op.profile_read()
    op.profile(False)
    _, mu, lam, _, shr = op.ita_solve_safeguarded(y, bits, k, iters, c=c, kappa=kappa,
                                                  max_shrinks=max_shrinks, out=out, ws=ws)
    shr = shr.cpu()
    return {
        "workload": f"the same scene, k = {k}, c = {c}, kappa = {kappa}, at most {max_shrinks} shrinks "
                    f"per iteration, {iters} iterations per step",
        "iterations_per_s": steps * iters / t,
        "shrinks_total": int(shr.sum()),
        "iterations_with_shrinks": int((shr > 0).sum()),
        "passes_avg_us": {kind: 1e3 * ms / cnt for kind, (ms, cnt) in prof.items()},
        "passes_launches": {kind: cnt for kind, (ms, cnt) in prof.items()},
        "mu_last": float(mu[-1]), "lambda_last": float(lam[-1]),
    }


def bench_rda(shape, y, bits, lam, iters, steps, device):
    """The fixed-parameter iteration with the range-Doppler operator of
    eq. (RDA) (8-tap truncated-sinc migration correction) on the headline
    scene: iterations/s and the average duration of each pass kind."""
    import torch
    import inputs
    import paper_1302_3120_amd as pk
    op = pk.make_operator(inputs.RADAR_STRIPMAP, shape, chain="rda", taps=8)
    out = torch.empty_like(y)
    ws = op.workspace(1, device)

    def step():
        op.ita_solve(y, bits, lam, iters, out=out, ws=ws)

    t = time_steps(step, steps, 1)
    op.profile(True)
    op.profile_read()
    step()
    prof = op.profile_read()
    op.profile(False)
    return {
        "workload": f"the same scene and lambda, range-Doppler G and M (8 taps), {iters} iterations per step",
        "iterations_per_s": steps * iters / t,
        "passes_avg_us": {kind: 1e3 * ms / cnt for kind, (ms, cnt) in prof.items()},
    }


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


def cpu_baseline(shape, seed, iters=3):
    """The FP64 oracle, as it stands, on the host: ``iters`` full ITA
    iterations (G, M and the threshold) on the same workload shape."""
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
    ita.ita(y, mask, 0.5, iters, g, x0=x1)  # iterations from a non-zero iterate
    dt = time.perf_counter() - t0
    return dict(value=iters / dt, unit="iterations/s", cores=threads, kind="oracle",
                sample=f"{iters} ITA iterations (G + G^H + soft threshold, naive FP64 DFTs "
                       f"as matrix products) on a {shape[0]}x{shape[1]} scene, 50% mask; "
                       f"{dt:.1f} s")


def kernel_source_digest():
    """SHA-256 over the HIP kernel sources: counter figures taken from an
    older version of the kernels are not reported."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1302_3120_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def copy_calibration(device, reps=3):
    """A plain device-to-device copy of CAL_MIB MiB, for scaling the HBM byte
    counters: it reads and writes exactly CAL_MIB MiB per dispatch."""
    import torch
    n = CAL_MIB * 2 ** 20 // 4
    src = torch.ones(n, dtype=torch.float32, device=device)
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()


def _rows(pattern):
    out = []
    for f in sorted(glob.glob(pattern, recursive=True)):
        with open(f, newline="") as fh:
            out.extend(csv.DictReader(fh))
    return out


def sq_summary(sq_dirs, n, kinds):
    """Per-kernel medians of the SQ counters of one or more rocprofv3 --pmc
    runs, and what follows from them: VALU instructions per element
    (SQ_INSTS_VALU counts wave instructions: x 64 lanes / n elements), the
    time the SIMDs need to issue them (4 cycles per wave instruction on a
    16-lane SIMD, 1024 SIMDs at 2.4 GHz) and the share of wave time spent
    waiting (SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES)."""
    vals = {}
    for d in sq_dirs:
        for r in _rows(os.path.join(d, "**", "*counter_collection.csv")):
            if not r["Counter_Name"].startswith("SQ_"):
                continue
            vals.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(
                float(r["Counter_Value"]))
    lines = ["", "## SQ counters per dispatch (--pmc SQ_*; medians)", ""]
    names = sorted({c for k in vals.values() for c in k})
    lines += ["| kernel | " + " | ".join(names) + " | VALU instr / element | VALU issue us "
              "at 2.4 GHz | wait share |", "|---" * (len(names) + 4) + "|"]
    for kind in kinds:
        sym = kind_symbol(kind, n)
        ks = [k for k in vals if sym in k]
        if not ks:
            continue
        c = {name: statistics.median(v) for name, v in vals[ks[0]].items()}
        valu = c.get("SQ_INSTS_VALU")
        per_el = "%.1f" % (valu * 64.0 / (n * n)) if valu else "-"
        issue = "%.1f" % (valu * 4.0 / (1024 * 2.4e9) * 1e6) if valu else "-"
        wait = ("%.2f" % (c["SQ_WAIT_INST_ANY"] / c["SQ_WAVE_CYCLES"])
                if c.get("SQ_WAIT_INST_ANY") and c.get("SQ_WAVE_CYCLES") else "-")
        lines.append("| %s (%s) | " % (kind, sym) + " | ".join("%.4g" % c.get(nm, float("nan"))
                                                          for nm in names) +
                     " | %s | %s | %s |" % (per_el, issue, wait))
    return lines


def rocprof_summary(stats_dir, fetch_dir, write_dir, n, command, title="ITA passes", sq_dirs=()):
    """Text summary of rocprofv3 output: per-kernel durations (kernel-trace
    --stats) and per-dispatch HBM bytes (FETCH_SIZE and WRITE_SIZE runs, each
    scaled so that the calibration copy reads and writes CAL_MIB MiB).  With
    fetch_dir "-" only the durations (all kernels)."""
    lines = ["# rocprofv3 summary: %s at %dx%d complex64" % (title, n, n), "",
             "Commands (from the repository root, on one MI355X):", ""]
    lines += ["    " + c for c in command]
    lines += ["", "## Kernel durations (--kernel-trace --stats)", "",
              "| kernel | calls | average us | min us | max us | % of GPU time |",
              "|---|---|---|---|---|---|"]
    stats = sorted(_rows(os.path.join(stats_dir, "**", "*kernel_stats.csv")),
                   key=lambda r: -float(r["Percentage"]))
    for r in stats[:8] if fetch_dir != "-" else stats:
        if fetch_dir == "-" and float(r["Percentage"]) < 0.05:
            continue
        name = r["Name"] if len(r["Name"]) <= 90 else r["Name"][:87] + "..."
        lines.append("| %s | %s | %.1f | %.1f | %.1f | %.2f |" % (
            name, r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    if fetch_dir == "-":
        return "\n".join(lines) + "\n"
    per = {}
    for d, counter in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        groups = {}
        for r in _rows(os.path.join(d, "**", "*counter_collection.csv")):
            if r["Counter_Name"] != counter:
                continue
            groups.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        # the runtime's buffer copy (torch's copy_ of contiguous tensors),
        # else any copy kernel: elementwise copies of the scene set-up can be
        # larger than the calibration copy at 8192 x 8192
        copies = {k: v for k, v in groups.items() if "copybuffer" in k.lower()}
        if not copies:
            copies = {k: v for k, v in groups.items() if "copy" in k.lower()}
        if not copies:
            raise SystemExit("no copy kernel in " + d)
        # the calibration copy is the largest copy dispatch of the run
        cal_name = max(copies, key=lambda k: max(copies[k]))
        cal_kib = max(copies[cal_name])
        factor = CAL_MIB * 1024.0 / cal_kib
        per[counter] = (factor, cal_name, cal_kib,
                        {k: (len(v), statistics.median(v)) for k, v in groups.items()})
    lines += ["", "## HBM bytes per dispatch (--pmc FETCH_SIZE; --pmc WRITE_SIZE)", ""]
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        factor, cal_name, cal_kib, _ = per[counter]
        short = cal_name if len(cal_name) <= 60 else cal_name[:57] + "..."
        lines.append("- %s calibration: torch's device copy `%s` of %d MiB counts %.1f KiB per "
                     "dispatch; scale factor %.4f" % (counter, short, CAL_MIB, cal_kib, factor))
    lines += ["", "| kernel | dispatches | FETCH_SIZE KiB (median) | WRITE_SIZE KiB (median) "
                  "| fetch MB (scaled) | write MB (scaled) |", "|---|---|---|---|---|---|"]
    fetch_groups = per["FETCH_SIZE"][3]
    write_groups = per["WRITE_SIZE"][3]
    machine = []
    for kind in KIND_SYMBOL:
        sym = kind_symbol(kind, n)
        fk = [k for k in fetch_groups if sym in k]
        wk = [k for k in write_groups if sym in k]
        if not fk or not wk:
            continue
        cnt, f_kib = fetch_groups[fk[0]]
        _, w_kib = write_groups[wk[0]]
        fb = f_kib * 1024 * per["FETCH_SIZE"][0]
        wb = w_kib * 1024 * per["WRITE_SIZE"][0]
        if True:
            lines.append("| %s | %d | %.1f | %.1f | %.1f | %.1f |" % (
                fk[0], cnt, f_kib, w_kib, fb / 1e6, wb / 1e6))
        machine.append("traffic %s %.0f %.0f" % (kind, fb, wb))
    lines += ["", "Algorithmic bytes per dispatch: 16 B/pixel (row passes), 24 B/pixel (residual "
                  "column pass), 16 + 24 x (nonzero fraction) B/pixel (update pass of the "
                  "sparse iterate), 24.125 B/pixel (first column pass: y, mask, two outputs).", "",
              "Machine-readable lines (kind, fetch bytes, write bytes per dispatch, scaled):", ""]
    lines += ["    " + m for m in machine]
    lines += ["    kernel_sources_sha256 " + kernel_source_digest(), ""]
    if sq_dirs:
        lines += sq_summary(sq_dirs, n, list(KIND_SYMBOL))
    return "\n".join(lines) + "\n"


def marker_summary(marker_dir, n, command):
    """Text summary of the library's roctx ranges (rocprofv3 --marker-trace)."""
    lines = ["# roctx ranges of one solve at %dx%d complex64 (rocprofv3 --marker-trace)" % (n, n), "",
             "Command (from the repository root, on one MI355X):", ""]
    lines += ["    " + c for c in command]
    lines += ["", "The library pushes a named host range around each entry point (`cssar_ita_solve`, "
                  "`cssar_apply_G`, ...) and",
              "around each pass launch (`cssar row M`, `cssar col residual`, ...).  The ranges time "
              "the host side of",
              "the call (argument checks and the asynchronous launches), not the kernels: the kernel "
              "trace of the same",
              "run gives those.", "",
              "| range | calls | total us | average us | min us | max us |", "|---|---|---|---|---|---|"]
    rows = sorted(_rows(os.path.join(marker_dir, "**", "*marker_api_stats.csv")),
                  key=lambda r: -float(r["TotalDurationNs"]))
    for r in rows:
        lines.append("| %s | %s | %.1f | %.1f | %.1f | %.1f |" % (
            r["Name"], r["Calls"], float(r["TotalDurationNs"]) / 1e3, float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3))
    return "\n".join(lines) + "\n"


def load_traffic():
    """Per-kind scaled HBM bytes per dispatch from the committed summary, or
    None when it is missing or the kernel sources changed since."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    out, digest = {}, None
    for line in text.splitlines():
        w = line.split()
        if len(w) == 4 and w[0] == "traffic":
            out[w[1]] = float(w[2]) + float(w[3])
        elif len(w) == 2 and w[0] == "kernel_sources_sha256":
            digest = w[1]
    if digest != kernel_source_digest():
        return None
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=100, help="ITA iterations per step")
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 64-scene batched-versus-plain-loop measurement")
    ap.add_argument("--no-adaptive", action="store_true",
                    help="skip the adaptive step-and-threshold measurement")
    ap.add_argument("--no-safeguard", action="store_true",
                    help="skip the safeguarded adaptive solve measurement")
    ap.add_argument("--no-rda", action="store_true",
                    help="skip the range-Doppler operator measurement")
    ap.add_argument("--no-grad", action="store_true",
                    help="skip the differentiated (forward + reverse pass) measurement")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the event-instrumented region (plain timing only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help=f"also run a {CAL_MIB} MiB device copy (for counter calibration)")
    ap.add_argument("--rocprof-summary", nargs=3, metavar=("STATS_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="print a text summary of rocprofv3 output and exit (no GPU)")
    ap.add_argument("--command", action="append", default=[],
                    help="command line recorded in the --rocprof-summary text")
    ap.add_argument("--summary-title", default="ITA passes",
                    help="title of the --rocprof-summary text")
    ap.add_argument("--sq-dir", action="append", default=[],
                    help="rocprofv3 --pmc SQ_* output directories for the --rocprof-summary text")
    ap.add_argument("--marker-summary", metavar="MARKER_DIR",
                    help="print a text summary of the roctx ranges of a rocprofv3 --marker-trace run")
    args = ap.parse_args()

    if args.marker_summary:
        print(marker_summary(args.marker_summary, args.size, args.command))
        return
    if args.rocprof_summary:
        print(rocprof_summary(*args.rocprof_summary, args.size, args.command, args.summary_title,
                              args.sq_dir))
        return

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the single-scene "
                                   "ITA is not sharded across GPUs (--gpus must be 1)"}))
        sys.exit(2)

    import torch
    import paper_1302_3120_amd as pk
    import inputs

    dev = torch.device("cuda:0")
    shape = (args.size, args.size)
    # the sparse recipe of the headline scene; its own record (seed) where the
    # grid has one (the wide-swath 8192 x 8192 scene)
    wl = inputs.workload(f"sparse_{args.size}" if f"sparse_{args.size}" in inputs.WORKLOADS
                         else "sparse_4096")
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
    # the median of five further timed repeats, beside the single timed region
    # of exactly --steps steps
    reps = [args.iters * max(1, args.steps // 2) / time_steps(step, max(1, args.steps // 2), 0)
            for _ in range(5)]
    nnz_frac = float(torch.count_nonzero(out)) / n
    PASS_BYTES["col_update_sparse"] = sparse_update_bytes(nnz_frac)
    moved = PASS_BYTES["row_G"] + PASS_BYTES["col_residual"] + PASS_BYTES["row_M"] + \
        PASS_BYTES["col_update_sparse"]
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
        "repeats_median_iterations_per_s": statistics.median(reps),
        "repeats_iterations_per_s": reps,
        # the sparse iterate moves fewer bytes than the 80.125 B/pixel of the
        # conventional figure: the iteration's own algorithmic bytes
        "iterate_nonzero_fraction": nnz_frac,
        "iteration_bytes_per_pixel": moved,
        "hbm_frac_iteration_bytes": moved * n * its / (HBM_PEAK_GBS * 1e9),
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
        # The dominant kernel is the symbol with the most GPU time: the row
        # passes of M and G are one kernel and are counted together.
        by_sym = {}
        for kind, kd in kernels.items():
            sym = kind_symbol(kind, shape[1] if kind.startswith("row") else shape[0])
            agg = by_sym.setdefault(sym, {"kinds": [], "ms": 0.0, "cnt": 0, "algo_GB": kd["algo_GB"]})
            agg["kinds"].append(kind)
            agg["ms"] += kd["total_ms"]
            agg["cnt"] += kd["launches"]
        dom = max(by_sym, key=lambda k: by_sym[k]["ms"])
        agg = by_sym[dom]
        avg_us = 1e3 * agg["ms"] / agg["cnt"]
        gbs = agg["algo_GB"] / (avg_us * 1e-6)
        traffic = load_traffic() if shape == (4096, 4096) else None
        rec["roofline"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": gbs / HBM_PEAK_GBS,
                           "traffic": traffic.get(agg["kinds"][0]) if traffic else None,
                           "kernel": dom, "pass_kinds": agg["kinds"], "avg_us": avg_us,
                           "launches": agg["cnt"], "algorithmic_bytes": agg["algo_GB"] * 1e9}
        rec["kernels"] = kernels
        rec["profiled_region_iterations_per_s"] = args.steps * args.iters / dt2

    if args.copy_calibration:
        copy_calibration(dev)

    if not args.no_adaptive:
        log("bench: adaptive step and threshold")
        rec["adaptive"] = bench_adaptive(op, y, bits, k, args.iters, 3, dev)

    if not args.no_safeguard:
        log("bench: safeguarded adaptive solve")
        rec["safeguarded"] = bench_safeguarded(op, y, bits, k, args.iters, 3, dev)

    if not args.no_rda:
        log("bench: range-Doppler operator")
        rec["range_doppler"] = bench_rda(shape, y, bits, lam, args.iters, 3, dev)

    if not args.no_batched:
        rec["batched"] = bench_batched(3, args.iters, dev)

    if not args.no_grad:
        rec["differentiated"] = bench_grad(5, dev)

    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on the host (three iterations)")
        rec["cpu_baseline"] = cpu_baseline(shape, 1234)

    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
