#!/usr/bin/env python3
"""Benchmark of the MPA hot path on one MI355X.

One step = one DM period (z -> z + 1) of the 8-channel WDM workload: 2^18
modes, FP32 node evaluations with FP64-built phases and FP64 carry, 4096-point
blocks with 512-point halos, long step L = 2.5e-4 with M = 2 intervals and 2
Picard sweeps, i.e. 4000 launches of the fused long-step kernel per step.

Printed (one JSON line on stdout):
  value        MPA mode-steps/s = N * (dz intervals advanced) / wall time
  roofline     the fused long-step kernel against the FP32 vector peak
               (algorithmic flops per launch / average launch time, HIP events)
  cpu_baseline the FP64 oracle on the host, on a bounded sample
  accuracy     rel-L2 error after one DM period against an FP64 reference
               (Richardson-extrapolated fine FP64 split-step on the GPU)
  split_step   the GPU split-step comparator at equal or better accuracy
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("paper_1101_0086_amd/csrc/mpa_kernels.hip", "paper_1101_0086_amd/csrc/long_step_body.inc",
                  "paper_1101_0086_amd/csrc/block_fft.hpp", "paper_1101_0086_amd/csrc/cx.hpp")
PMC_PROFILE = "profiles/mpa_block_kernel_wdm8_n262144_pmc.md"


def measured_traffic(config: str):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    PMC summary (FETCH_SIZE and WRITE_SIZE, calibrated on a copy of known
    size), or None when the kernel sources or the launch configuration
    (`config`, e.g. "B=4096 H=512 L=0.00025 M=4 n_iter=2") changed since it
    was taken."""
    import hashlib
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    try:
        text = open(os.path.join(ROOT, PMC_PROFILE)).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.startswith(("traffic_bytes_per_launch:", "kernel-source-sha256:", "launch-config:")))
    if fields.get("kernel-source-sha256", "").strip() != h.hexdigest():
        return None
    if fields.get("launch-config", "").strip() != config:
        return None
    return float(fields["traffic_bytes_per_launch"])


def flops_per_block(B: int, M: int, n_iter: int) -> float:
    """Algorithmic flops of one block in one long step: 5 B log2 B per
    transform for (3 + 2 n M) transforms (FP64 carry in and out, node 0, and
    two per node and sweep), 35 flops per point per node and sweep (phase and
    conjugate phase products, scale, |A|^2 A, compensated trapezoid update)
    and 15 per point for gather and reconstruction."""
    return 5.0 * B * math.log2(B) * (3 + 2 * n_iter * M) + B * (35.0 * n_iter * M + 15.0)


def cpu_baseline(w, budget_s: float = 12.0):
    """The FP64 oracle (blocked MPA, numpy, one thread) on long steps of the
    same workload until the budget is spent; mode-steps/s."""
    import oracle as O
    a = w.field()
    s = w.mpa
    t0 = time.perf_counter()
    steps = 0
    while True:
        a = O.mpa_step(a, w.grid.dt, w.dmmap, s.L, s.M, s.n_iter, steps, s.block, s.halo)
        steps += 1
        el = time.perf_counter() - t0
        if el > budget_s or steps >= 400:
            break
    return {"value": w.grid.n * s.M * steps / el, "unit": "mode-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} long steps (L={s.L}, M={s.M}) of the same 2^18-mode field, "
                      f"{el:.1f} s, numpy FFT single thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="wdm8_n262144_f32")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-compare", action="store_true", help="skip accuracy and split-step comparison")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 256-instance measurement")
    ap.add_argument("--no-grad", action="store_true", help="skip the gradient (reverse pass) measurement")
    ap.add_argument("--grad-periods", type=int, default=20, help="map periods of the gradient measurement")
    ap.add_argument("--block", type=int, help="override the workload's block size")
    ap.add_argument("--halo", type=int, help="override the workload's halo")
    ap.add_argument("--long-step", type=float, help="override the workload's long step L")
    ap.add_argument("--nodes", type=int, help="override the workload's nodes per long step M")
    ap.add_argument("--pmc-grad", action="store_true",
                    help="for rocprofv3 --pmc: 20 reverse long steps of the 2^16-mode gradient workload")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="for rocprofv3 --pmc: a 64 MiB copy (counter calibration), then 20 long steps")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this implementation runs on one GPU; --gpus must be 1 "
              "(the multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1101_0086_amd as P
    from workloads import WORKLOADS

    if args.pmc_grad:
        g = WORKLOADS["wdm4_n65536_f32"]
        gs = g.mpa
        pl = P.MPAPlan(g.grid.n, g.grid.dt, g.dmmap, gs.L, gs.M, gs.n_iter, gs.block, gs.halo, P.MPA_C64,
                       gs.omega_band)
        xg = torch.from_numpy(g.field()).to(device="cuda:0", dtype=torch.complex64)
        ck = pl.propagate_checkpointed(xg, 0.0, 20 * gs.L)
        pl.adjoint(ck, (2 * xg).contiguous(), 0.0, 20 * gs.L)
        torch.cuda.synchronize()
        pl.close()
        print(json.dumps({"pmc_grad": True, "reverse_launches": 20}), flush=True)
        return

    w = WORKLOADS[args.workload]
    over = {k: v for k, v in (("block", args.block), ("halo", args.halo), ("L", args.long_step),
                              ("M", args.nodes)) if v is not None}
    if over:                # another launch configuration of the same workload
        import dataclasses
        w = dataclasses.replace(w, mpa=dataclasses.replace(w.mpa, **over))
    s = w.mpa
    n = w.grid.n
    launches_per_step = int(round(1.0 / s.L))
    log(f"workload {w.name}: N={n} B={s.block} H={s.halo} L={s.L} M={s.M} n_iter={s.n_iter}")
    a0 = w.field()
    prec = P.MPA_C64 if w.precision == "f32" else P.MPA_C128
    cdt = torch.complex64 if prec == P.MPA_C64 else torch.complex128
    plan = P.MPAPlan(n, w.grid.dt, w.dmmap, s.L, s.M, s.n_iter, s.block, s.halo, prec, s.omega_band)
    info = plan.info()
    x = torch.from_numpy(a0).to(device="cuda:0", dtype=cdt)

    if args.pmc_pass:
        big = torch.zeros(1 << 23, dtype=torch.complex64, device="cuda:0")     # 64 MiB
        torch.cuda.synchronize()
        copy = big.clone()                  # one copy kernel: reads 64 MiB, writes 64 MiB
        torch.cuda.synchronize()
        plan.propagate(x, 0.0, 20 * s.L)
        torch.cuda.synchronize()
        del copy
        print(json.dumps({"pmc_pass": True, "copy_bytes": 1 << 26, "launches": 20}), flush=True)
        plan.close()
        return

    z = 0.0
    for _ in range(args.warmup):
        plan.propagate(x, z, z + 1.0)
        z += 1.0
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        plan.propagate(x, z, z + 1.0)
        z += 1.0
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    mode_steps = n * s.M * launches_per_step * args.steps
    value = mode_steps / wall
    launch_s = gpu_ms * 1e-3 / (launches_per_step * args.steps)
    fl = flops_per_block(info["block"], s.M, s.n_iter) * info["n_blocks"]
    achieved = fl / launch_s / 1e12
    log(f"MPA: {value:.3e} mode-steps/s, {launch_s * 1e6:.2f} us per long-step launch, "
        f"{achieved:.2f} TFLOP/s algorithmic")
    out = {
        "metric": "mode-steps/s, MPA vs split-step, 1 MI355X, at stated rel-L2 error vs FP64",
        "value": value, "unit": "mode-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "n_modes": n, "channels": w.n_channels,
                   "modulation": w.modulation, "block": info["block"], "halo": info["halo"],
                   "n_blocks": info["n_blocks"], "L": s.L, "M": s.M, "n_iter": s.n_iter,
                   "step": f"one DM period = {launches_per_step} long steps",
                   "precision": "FP32 node work, FP64 phases and carry"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": measured_traffic(f"B={s.block} H={s.halo} L={s.L:g} M={s.M} n_iter={s.n_iter}")
                     if w.name == "wdm8_n262144_f32" else None,
                     "kernel": "mpa_block_kernel", "launch_us": launch_s * 1e6,
                     "flops_per_launch": fl},
    }

    if not args.no_compare:
        out.update(compare(w, a0, plan, x, torch, P))
    if not args.no_batch:
        out["batched"] = batched(torch, P)
        out["autotune"] = autotune_table(w, a0, torch, P)
        out["large"] = large(torch, P)
    if not args.no_grad:
        out["gradient"] = gradient(torch, P, args.grad_periods)
        out["batched_gradient"] = batched_gradient(torch, P)
    plan.close()
    if not args.no_cpu:
        log("CPU oracle baseline ...")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


def batched(torch, P, count=256, steps=200):
    """256 independent fields, N uniform over 2^14..2^18, 1-16 channels,
    sigma uniform in [0.5, 2], 4096-blocks with 512-halos, L = 5e-5, M = 1,
    2 sweeps: one launch per long step for all instances, eager and as a
    replayed HIP graph of `steps` long steps."""
    import numpy as np
    from workloads import dm_map
    from workloads.wdm import batched_instances
    inst = batched_instances(count, 4)
    ns = [g.n for g, _, _, _ in inst]
    sig = [s for _, _, s, _ in inst]
    dt = inst[0][0].dt
    band = 0.5 * 15 * 40.0 + 5.0
    L, M, nit = 5e-5, 1, 2
    bp = P.MPABatchPlan(ns, dt, dm_map(beta3=0.1), L, M, nit, 4096, 512, P.MPA_C64, band, sigma_scale=sig)
    info = bp.info()
    x = torch.from_numpy(np.concatenate([f for _, _, _, f in inst])).to(device="cuda:0", dtype=torch.complex64)
    z1 = steps * L
    bp.propagate(x, 0.0, z1)                        # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bp.propagate(x, 0.0, z1)
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t0
    g = bp.capture(x, 0.0, z1)
    g.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.launch()
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    g.close()
    bp.close()
    ms = info["total_samples"] * M * steps
    log(f"batched: {info['work_items']} work items, eager {ms / t_eager:.3e}, graph {ms / t_graph:.3e} mode-steps/s")
    # block size and overlap at the same dz (candidates of the autotuner for the
    # shortest instance), each timed eagerly over the same distance
    from paper_1101_0086_amd.autotune import candidates
    dz = L / M
    tuned = []
    for c in candidates(min(ns), dt, dm_map(beta3=0.1), dz, band):
        cp = P.MPABatchPlan(ns, dt, dm_map(beta3=0.1), c.L, c.M, nit, c.block, c.halo, P.MPA_C64, band,
                            sigma_scale=sig)
        y = x.clone()
        cp.propagate(y, 0.0, 4 * c.L)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cp.propagate(y, 0.0, z1)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        cp.close()
        tuned.append({"block": c.block, "halo": c.halo, "L": c.L, "M": c.M,
                      "mode_steps_per_s": info["total_samples"] * (z1 / dz) / el})
    log("batched, block size and overlap at dz = %.1e: " % dz
        + ", ".join(f"B={t['block']} H={t['halo']} M={t['M']}: {t['mode_steps_per_s']:.3e}" for t in tuned))
    return {"instances": count, "total_modes": info["total_samples"], "work_items_per_launch": info["work_items"],
            "L": L, "M": M, "n_iter": nit, "block": 4096, "halo": 512, "long_steps": steps,
            "mode_steps_per_s_eager": ms / t_eager, "mode_steps_per_s_graph": ms / t_graph,
            "us_per_long_step_graph": t_graph / steps * 1e6, "block_overlap_at_same_dz": tuned}


def autotune_table(w, a0, torch, P):
    """Autotuner over (block, halo, L, M) at the workload's dz (fixed accuracy)."""
    from paper_1101_0086_amd.autotune import autotune
    s = w.mpa
    x = torch.from_numpy(a0).to(device="cuda:0", dtype=torch.complex64)
    best, cands = autotune(x, w.grid.dt, w.dmmap, s.L / s.M, s.n_iter, s.omega_band)
    rows = [{"block": c.block, "halo": c.halo, "L": c.L, "M": c.M,
             "mode_steps_per_s": w.grid.n / (c.seconds_per_unit_z * (s.L / s.M))} for c in cands]
    log("autotune: " + ", ".join(f"B={r['block']} H={r['halo']} L={r['L']:.2e} M={r['M']}: {r['mode_steps_per_s']:.3e}"
                                 for r in rows))
    return {"dz": s.L / s.M, "candidates": rows, "best_block": best.block, "best_halo": best.halo}


def large(torch, P, steps=200):
    """The 32-channel QPSK workload (2^22 modes, 1366 blocks of 4096): MPA
    (L = dz = 7.8125e-6, 2 sweeps) and split-step at the same dz, throughput
    over `steps` long steps from the seeded field (no accuracy run: the
    channel band reaches half the grid's Nyquist frequency), and the
    autotuner's table of block sizes and overlaps at that dz."""
    from workloads import WORKLOADS
    w = WORKLOADS["wdm32_n4194304_f32"]
    s = w.mpa
    a = w.field()
    plan = P.MPAPlan(w.grid.n, w.grid.dt, w.dmmap, s.L, s.M, s.n_iter, s.block, s.halo, P.MPA_C64, s.omega_band)
    x = torch.from_numpy(a).to(device="cuda:0", dtype=torch.complex64)
    plan.propagate(x, 0.0, 4 * s.L)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.propagate(x, 0.0, steps * s.L)
    torch.cuda.synchronize()
    t_mpa = time.perf_counter() - t0
    nb = plan.info()["n_blocks"]
    plan.close()
    dz = s.L / s.M
    ss = P.SSPlan(w.grid.n, w.grid.dt, w.dmmap, dz, P.MPA_C64)
    y = torch.from_numpy(a).to(device="cuda:0", dtype=torch.complex64)
    ss.propagate(y, 0.0, 4 * dz)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ss.propagate(y, 0.0, steps * dz)
    torch.cuda.synchronize()
    t_ss = time.perf_counter() - t0
    ss.close()
    n = w.grid.n
    # block size and overlap autotuned at the same dz
    from paper_1101_0086_amd.autotune import autotune
    x = torch.from_numpy(a).to(device="cuda:0", dtype=torch.complex64)
    pick, cands = autotune(x, w.grid.dt, w.dmmap, dz, s.n_iter, s.omega_band, launches=20)
    tuned = [{"block": c.block, "halo": c.halo, "L": c.L, "M": c.M,
              "mode_steps_per_s": n / (c.seconds_per_unit_z * dz)} for c in cands]
    r = {"workload": w.name, "n_modes": n, "n_blocks": nb, "dz": dz,
         "mpa_mode_steps_per_s": n * s.M * steps / t_mpa, "mpa_us_per_launch": t_mpa / steps * 1e6,
         "ss_f32_mode_steps_per_s": n * steps / t_ss, "autotune": tuned,
         "autotune_pick": {"block": pick.block, "halo": pick.halo, "L": pick.L, "M": pick.M}}
    log(f"large: MPA {r['mpa_mode_steps_per_s']:.3e} ({r['mpa_us_per_launch']:.0f} us/launch), "
        f"split-step {r['ss_f32_mode_steps_per_s']:.3e} mode-steps/s; autotune: "
        + ", ".join(f"B={t['block']} H={t['halo']} M={t['M']}: {t['mode_steps_per_s']:.3e}" for t in tuned))
    return r


def adjoint_flops_per_block(B: int, M: int, n_iter: int) -> float:
    """Algorithmic flops of the reverse pass of one block and long step:
    4 n_iter M + 7 transforms (recomputed forward and reverse) of 5 B log2 B
    flops, and about 100 n_iter M + 60 flops per point of elementwise work."""
    return 5.0 * B * math.log2(B) * (4 * n_iter * M + 7) + B * (100.0 * n_iter * M + 60)


def gradient(torch, P, periods=20):
    """Gradient workload: 2^16 modes, 4 OOK channels, 20 map periods
    (80000 long steps, B = 2048, H = 256, L = 2.5e-4, M = 2, 2 sweeps, FP32
    node work), loss = sum |A(z1) - target|^2: the plain forward, the
    checkpointed forward (one checkpoint per period) and the reverse pass
    (which recomputes each period from its checkpoint, the next period's
    recompute overlapped with the current period's reverse launches), timed
    separately after a warm-up.  adjoint_tflops_wall: the reverse kernels'
    algorithmic flops over the reverse pass's wall time (a lower bound of the
    kernel rate)."""
    from workloads import WORKLOADS
    w = WORKLOADS["wdm4_n65536_f32"]
    s = w.mpa
    a = w.field()
    plan = P.MPAPlan(w.grid.n, w.grid.dt, w.dmmap, s.L, s.M, s.n_iter, s.block, s.halo, P.MPA_C64, s.omega_band)
    x0 = torch.from_numpy(a).to(device="cuda:0", dtype=torch.complex64)
    target = torch.from_numpy(w.field(seed=w.seed + 100)).to(device="cuda:0", dtype=torch.complex64)
    z1 = float(periods)
    steps = int(round(z1 / s.L))

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    x = x0.clone()
    ck = plan.propagate_checkpointed(x, 0.0, 20 * s.L)            # warm-up, workspace
    plan.adjoint(ck, (2 * x).contiguous(), 0.0, 20 * s.L)
    x = x0.clone()
    t_fwd, _ = timed(lambda: plan.propagate(x, 0.0, z1))
    x = x0.clone()
    t_ck, ck = timed(lambda: plan.propagate_checkpointed(x, 0.0, z1))
    g = (2 * (x - target)).contiguous()
    t_adj, pg = timed(lambda: plan.adjoint(ck, g, 0.0, z1))
    nb = plan.info()["n_blocks"]
    plan.close()
    fl = adjoint_flops_per_block(s.block, s.M, s.n_iter) * nb
    pgc = pg.cpu().numpy()
    r = {"workload": w.name, "n_modes": w.grid.n, "periods": periods, "long_steps": steps, "block": s.block,
         "halo": s.halo, "L": s.L, "M": s.M, "n_iter": s.n_iter, "n_blocks": nb, "checkpoints": int(ck.shape[0]),
         "forward_s": t_fwd, "checkpointed_forward_s": t_ck, "reverse_s": t_adj,
         "gradient_over_forward": (t_ck + t_adj) / t_fwd,
         "gradient_mode_steps_per_s": w.grid.n * s.M * steps / (t_ck + t_adj),
         "reverse_us_per_long_step": t_adj / steps * 1e6,
         "adjoint_flops_per_launch": fl,
         "adjoint_tflops_wall": fl * steps / t_adj / 1e12,
         "dl_dsigma": pgc[0].tolist(), "dl_dbeta2": pgc[1].tolist(), "dl_dbeta3": pgc[2].tolist()}
    log(f"gradient ({periods} periods): forward {t_fwd:.2f} s, checkpointed {t_ck:.2f} s, reverse {t_adj:.2f} s "
        f"({r['gradient_over_forward']:.2f}x forward), reverse {r['reverse_us_per_long_step']:.1f} us per long step")
    # block size and overlap at the same dz: gradient over one period each
    from paper_1101_0086_amd.autotune import candidates
    dz = s.L / s.M
    table = []
    for c in candidates(w.grid.n, w.grid.dt, w.dmmap, dz, s.omega_band):
        pl = P.MPAPlan(w.grid.n, w.grid.dt, w.dmmap, c.L, c.M, s.n_iter, c.block, c.halo, P.MPA_C64, s.omega_band)
        x = x0.clone()
        ck = pl.propagate_checkpointed(x, 0.0, 20 * c.L)
        pl.adjoint(ck, (2 * x).contiguous(), 0.0, 20 * c.L)
        x = x0.clone()
        tc, ck = timed(lambda: pl.propagate_checkpointed(x, 0.0, 1.0))
        g = (2 * (x - target)).contiguous()
        ta, _ = timed(lambda: pl.adjoint(ck, g, 0.0, 1.0))
        pl.close()
        del ck
        table.append({"block": c.block, "halo": c.halo, "L": c.L, "M": c.M, "gradient_s_per_period": tc + ta,
                      "gradient_mode_steps_per_s": w.grid.n / dz / (tc + ta)})
    r["block_overlap_at_same_dz"] = table
    log("gradient, block size and overlap at dz = %.2e, one period: " % dz
        + ", ".join(f"B={t['block']} H={t['halo']} M={t['M']}: {t['gradient_s_per_period'] * 1e3:.0f} ms"
                    for t in table))
    return r


def batched_gradient(torch, P, count=32, periods=1):
    """Gradients of 32 instances of the 2^16-mode 4-channel workload (seeds
    differ, sigma scales uniform in [0.8, 1.2]) through one map period (4000
    long steps) with one batched launch per long step: checkpointed forward
    and reverse pass, timed after a warm-up, against the plain batched
    forward."""
    import numpy as np
    from workloads import WORKLOADS
    w = WORKLOADS["wdm4_n65536_f32"]
    s = w.mpa
    rng = np.random.default_rng(7)
    sig = rng.uniform(0.8, 1.2, count).tolist()
    ns = [w.grid.n] * count
    bp = P.MPABatchPlan(ns, w.grid.dt, w.dmmap, s.L, s.M, s.n_iter, s.block, s.halo, P.MPA_C64, s.omega_band,
                        sigma_scale=sig)
    info = bp.info()
    x0 = torch.from_numpy(np.concatenate([w.field(seed=w.seed + i) for i in range(count)])).to(
        device="cuda:0", dtype=torch.complex64)
    z1 = float(periods)
    steps = int(round(z1 / s.L))

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    x = x0.clone()
    ck = bp.propagate_checkpointed(x, 0.0, 20 * s.L)              # warm-up, workspace
    bp.adjoint(ck, (2 * x).contiguous(), 0.0, 20 * s.L)
    x = x0.clone()
    t_fwd, _ = timed(lambda: bp.propagate(x, 0.0, z1))
    x = x0.clone()
    t_ck, ck = timed(lambda: bp.propagate_checkpointed(x, 0.0, z1))
    g = (2 * x).contiguous()
    t_adj, _ = timed(lambda: bp.adjoint(ck, g, 0.0, z1))
    bp.close()
    ms = info["total_samples"] * s.M * steps
    r = {"workload": f"{count} x {w.name}", "total_modes": info["total_samples"],
         "work_items_per_launch": info["work_items"], "long_steps": steps,
         "forward_s": t_fwd, "checkpointed_forward_s": t_ck, "reverse_s": t_adj,
         "gradient_over_forward": (t_ck + t_adj) / t_fwd,
         "forward_mode_steps_per_s": ms / t_fwd,
         "gradient_mode_steps_per_s": ms / (t_ck + t_adj),
         "reverse_us_per_long_step": t_adj / steps * 1e6}
    log(f"batched gradient ({count} instances, {steps} long steps): forward {t_fwd:.2f} s, checkpointed "
        f"{t_ck:.2f} s, reverse {t_adj:.2f} s, gradient {r['gradient_mode_steps_per_s']:.3e} mode-steps/s")
    return r


def compare(w, a0, plan, x, torch, P):
    """Accuracy after one DM period and the split-step comparator at equal
    accuracy, both against a Richardson-extrapolated FP64 split-step
    reference computed on the GPU."""
    import numpy as np
    s = w.mpa
    n, dt = w.grid.n, w.grid.dt

    def run_ss(dz, prec, z1=1.0, timed=False):
        pl = P.SSPlan(n, dt, w.dmmap, dz, prec)
        cdt = torch.complex64 if prec == P.MPA_C64 else torch.complex128
        y = torch.from_numpy(a0).to(device="cuda:0", dtype=cdt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pl.propagate(y, 0.0, z1)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if timed:     # second run, warm
            y2 = torch.from_numpy(a0).to(device="cuda:0", dtype=cdt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pl.propagate(y2, 0.0, z1)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        pl.close()
        return y.cpu().numpy().astype(np.complex128), el

    log("FP64 reference (split-step, Richardson) ...")
    dz_ref = 0.5 / 64000
    r1, _ = run_ss(dz_ref, P.MPA_C128)
    r2, _ = run_ss(dz_ref / 2, P.MPA_C128)
    ref = (4 * r2 - r1) / 3
    ref_err = float(np.linalg.norm(r2 - ref) / np.linalg.norm(ref))

    omega = 2 * math.pi * np.fft.fftfreq(n, dt)
    band = np.abs(omega) <= s.omega_band + 50.0
    ref_band = np.fft.ifft(ref)[band]

    def err(a):
        """(full-band, in-band) relative L2 error; in-band keeps the channels'
        band plus 50, where blocked and full-window results are comparable
        (beyond it the grid aliases four-wave-mixing products)."""
        full = float(np.linalg.norm(a - ref) / np.linalg.norm(ref))
        inb = float(np.linalg.norm(np.fft.ifft(a)[band] - ref_band) / np.linalg.norm(ref_band))
        return full, inb

    y = torch.from_numpy(a0).to(device="cuda:0", dtype=x.dtype)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.propagate(y, 0.0, 1.0)
    torch.cuda.synchronize()
    t_mpa = time.perf_counter() - t0
    e_mpa_full, e_mpa = err(y.cpu().numpy().astype(np.complex128))
    log(f"MPA error after one period: in-band {e_mpa:.3e}, full-band {e_mpa_full:.3e} "
        f"(reference {ref_err:.1e}), {t_mpa * 1e3:.1f} ms")
    # the same long steps with fewer and more Picard sweeps (text after Eq. 7:
    # the iteration floor (L / z_nl)^(n+1) is far below the quadrature error here)
    picard = []
    for nit in (1, 3):
        pl = P.MPAPlan(n, dt, w.dmmap, s.L, s.M, nit, s.block, s.halo, P.MPA_C64, s.omega_band)
        y = torch.from_numpy(a0).to(device="cuda:0", dtype=x.dtype)
        pl.propagate(y, 0.0, 0.05)
        y = torch.from_numpy(a0).to(device="cuda:0", dtype=x.dtype)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pl.propagate(y, 0.0, 1.0)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        pl.close()
        e_full, e = err(y.cpu().numpy().astype(np.complex128))
        picard.append({"n_iter": nit, "rel_l2_in_band": e, "rel_l2_full_band": e_full, "seconds": el,
                       "mode_steps_per_s": n * s.M / s.L / el})
        log(f"MPA n_iter={nit}: in-band {e:.3e} full-band {e_full:.3e} time {el * 1e3:.1f} ms")
    # the autotuner's pick (block, halo, L, M) at the same quadrature interval
    from paper_1101_0086_amd.autotune import autotune
    dz_q = s.L / s.M
    pick, _ = autotune(torch.from_numpy(a0).to(device="cuda:0", dtype=x.dtype), dt, w.dmmap, dz_q, s.n_iter,
                       s.omega_band)
    pl = P.MPAPlan(n, dt, w.dmmap, pick.L, pick.M, s.n_iter, pick.block, pick.halo, P.MPA_C64, s.omega_band)
    y = torch.from_numpy(a0).to(device="cuda:0", dtype=x.dtype)
    pl.propagate(y, 0.0, 20 * pick.L)
    y = torch.from_numpy(a0).to(device="cuda:0", dtype=x.dtype)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pl.propagate(y, 0.0, 1.0)
    torch.cuda.synchronize()
    t_pick = time.perf_counter() - t0
    pl.close()
    e_full, e = err(y.cpu().numpy().astype(np.complex128))
    tuned = {"block": pick.block, "halo": pick.halo, "L": pick.L, "M": pick.M, "dz": dz_q,
             "rel_l2_in_band": e, "rel_l2_full_band": e_full, "seconds_one_period": t_pick,
             "mode_steps_per_s": n / dz_q / t_pick}
    log(f"autotuned pick B={pick.block} H={pick.halo} L={pick.L:.3e} M={pick.M}: in-band {e:.3e} "
        f"full-band {e_full:.3e}, {t_pick * 1e3:.1f} ms, {tuned['mode_steps_per_s']:.3e} mode-steps/s")
    # and the sweep count from the Picard residual for that pick (1e-5 of the
    # five-sweep result after 200 long steps, far below the quadrature error)
    from paper_1101_0086_amd.autotune import choose_n_iter
    nit_pick, dist = choose_n_iter(torch.from_numpy(a0).to(device="cuda:0", dtype=x.dtype), dt, w.dmmap,
                                   pick.L, pick.M, pick.block, pick.halo, s.omega_band)
    pl = P.MPAPlan(n, dt, w.dmmap, pick.L, pick.M, nit_pick, pick.block, pick.halo, P.MPA_C64, s.omega_band)
    y = torch.from_numpy(a0).to(device="cuda:0", dtype=x.dtype)
    pl.propagate(y, 0.0, 20 * pick.L)
    y = torch.from_numpy(a0).to(device="cuda:0", dtype=x.dtype)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pl.propagate(y, 0.0, 1.0)
    torch.cuda.synchronize()
    t_nit = time.perf_counter() - t0
    pl.close()
    e_full, e = err(y.cpu().numpy().astype(np.complex128))
    tuned["picard"] = {"n_iter": nit_pick, "residual_vs_five_sweeps": {str(k): v for k, v in dist.items()},
                       "rel_l2_in_band": e, "rel_l2_full_band": e_full, "seconds_one_period": t_nit,
                       "mode_steps_per_s": n / dz_q / t_nit}
    log(f"autotuned pick with n_iter={nit_pick} (Picard residual): in-band {e:.3e} full-band {e_full:.3e}, "
        f"{t_nit * 1e3:.1f} ms, {n / dz_q / t_nit:.3e} mode-steps/s")
    sweep = []
    best = None
    for k in (1000, 1414, 2000, 2828, 4000, 5657, 8000, 11314, 16000):
        dz = 0.5 / k
        for prec, label in ((P.MPA_C64, "f32"), (P.MPA_C128, "f64")):
            a, el = run_ss(dz, prec, timed=True)
            e_full, e = err(a)
            rec = {"dz": dz, "precision": label, "rel_l2_in_band": e, "rel_l2_full_band": e_full,
                   "seconds": el, "mode_steps_per_s": n * (1.0 / dz) / el}
            sweep.append(rec)
            log(f"SS {label} dz={dz:.3e}: in-band {e:.3e} full-band {e_full:.3e} time {el * 1e3:.1f} ms")
            if e <= e_mpa and (best is None or el < best["seconds"]):
                best = rec
    # blocking error at full size: FP64 blocked plan against the FP64 full-window
    # plan (four-step transforms, no blocks) after one period
    outs = {}
    for block, halo in ((0, 0), (s.block, s.halo)):
        pl = P.MPAPlan(n, dt, w.dmmap, s.L, s.M, s.n_iter, block, halo, P.MPA_C128, s.omega_band)
        y = torch.from_numpy(a0).to(device="cuda:0", dtype=torch.complex128)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pl.propagate(y, 0.0, 1.0)
        torch.cuda.synchronize()
        outs[block] = (y.cpu().numpy(), time.perf_counter() - t0)
        pl.close()
    fw, bl = np.fft.ifft(outs[0][0]), np.fft.ifft(outs[s.block][0])
    blocking = {"rel_l2_in_band": float(np.linalg.norm((bl - fw)[band]) / np.linalg.norm(fw[band])),
                "rel_l2_full_band": float(np.linalg.norm(outs[s.block][0] - outs[0][0]) / np.linalg.norm(outs[0][0])),
                "full_window_fp64_seconds": outs[0][1], "blocked_fp64_seconds": outs[s.block][1],
                "full_window_rel_l2_in_band_vs_reference": err(outs[0][0])[1]}
    log(f"blocking error after one period (FP64): in-band {blocking['rel_l2_in_band']:.2e}, "
        f"full-band {blocking['rel_l2_full_band']:.2e}; full window {outs[0][1] * 1e3:.0f} ms, "
        f"blocked {outs[s.block][1] * 1e3:.0f} ms")
    res = {"accuracy": {"mpa_rel_l2_in_band_after_one_period": e_mpa,
                        "mpa_rel_l2_full_band_after_one_period": e_mpa_full,
                        "in_band": f"|omega| <= {s.omega_band + 50.0:g}",
                        "reference": "FP64 split-step on the GPU at dz = "
                        f"{dz_ref:.3e} and dz/2, Richardson-extrapolated; the plain dz/2 run differs "
                        f"from it by {ref_err:.1e}",
                        "mpa_seconds_one_period": t_mpa},
           "picard_sweeps": picard,
           "autotuned_pick": tuned,
           "blocking_error": blocking,
           "split_step": {"sweep": sweep, "equal_accuracy": best,
                          "time_ratio_ss_over_mpa": (best["seconds"] / t_mpa) if best else None}}
    return res


if __name__ == "__main__":
    main()
