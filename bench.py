#!/usr/bin/env python3
"""Benchmark of the MPA hot path on one MI355X.

Headline workload: 32 QPSK channels, 2^22 modes, FP32 node evaluations with
FP64-built phases and FP64 carry; quadrature interval dz = 7.8125e-6 with
the block size, overlap and window shift the autotuner picks at that dz
(4096-point blocks, 1024-point halos, windows moved 192 samples against
their cores), long step L = 4 dz, 2 Picard sweeps.  One step = z -> z + 0.01
(320 launches of the fused long-step kernel, 1280 dz intervals).

Printed (one JSON line on stdout):
  value          MPA mode-steps/s = N * (dz intervals advanced) / wall time,
                 field resident in HBM
  roofline       the fused long-step kernel against the FP32 vector peak
                 (algorithmic flops per launch / average launch time from HIP
                 events over the timed region), with the effective-bandwidth
                 figure (one read and one write of the complex field per
                 node evaluation) beside it
  accuracy       rel-L2 error (in the channels' band and full band) after a
                 truncated distance against an FP64 split-step reference, the
                 split-step comparator swept over dz in both precisions, and
                 the split-step/MPA time ratio at equal accuracy
  cpu_baseline   the FP64 oracle on the host (blocked MPA, one thread, a
                 bounded sample), and the paper's own decomposition of a long
                 step over every host core
  ...            the single-channel FP64 2^12-mode workload, the 8-channel
                 2^18-mode workload, batches, autotuner tables, gradients
                 (extra keys)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3
HBM_PEAK_GBPS = 8000.0
HEADLINE = "wdm32_n4194304_f32"
STEP_Z = 0.01          # one bench step: z -> z + 0.01
ACC_Z = 0.025          # truncated distance of the accuracy runs


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("paper_1101_0086_amd/csrc/mpa_kernels.hip", "paper_1101_0086_amd/csrc/long_step_body.inc",
                  "paper_1101_0086_amd/csrc/block_fft.hpp", "paper_1101_0086_amd/csrc/cx.hpp")
PMC_PROFILE = "profiles/mpa_block_kernel_wdm32_n4194304_pmc.md"


def measured_traffic(config: str):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    PMC summary (FETCH_SIZE and WRITE_SIZE, calibrated on a copy of known
    size), or None when the kernel sources or the launch configuration
    (`config`) changed since it was taken."""
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
    conjugate phase products, scale, |A|^2 A, trapezoid update) and 15 per
    point for gather and reconstruction."""
    return 5.0 * B * math.log2(B) * (3 + 2 * n_iter * M) + B * (35.0 * n_iter * M + 15.0)


def host_cpu():
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def _plan(P, w, prec=None, **over):
    s = w.mpa
    kw = dict(L=s.L, M=s.M, n_iter=s.n_iter, block=s.block, halo=s.halo, shift=s.shift)
    kw.update(over)
    prec = P.MPA_C64 if prec is None else prec
    return P.MPAPlan(w.grid.n, w.grid.dt, w.dmmap, kw["L"], kw["M"], kw["n_iter"], kw["block"], kw["halo"], prec,
                     s.omega_band, shift=kw["shift"])


def _timed(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-compare", action="store_true", help="skip accuracy and split-step comparison")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 2^12- and 2^18-mode workloads, batches, autotuner tables and gradients")
    ap.add_argument("--grad-periods", type=int, default=20, help="map periods of the gradient measurement")
    ap.add_argument("--profile-pass", action="store_true",
                    help="for rocprofv3 --kernel-trace: 40 headline launches, 20 split-steps of each precision")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="for rocprofv3 --pmc: a 512 MiB copy (counter calibration), then 20 headline launches")
    ap.add_argument("--profile-large", action="store_true",
                    help="for rocprofv3 --kernel-trace: 10 long steps each of the 2^22-mode workload with "
                         "8192-blocks (H 1024, M 4) and 16384-blocks (H 4096, M 16), the autotuner's shapes")
    ap.add_argument("--pmc-grad", action="store_true",
                    help="for rocprofv3: 20 reverse long steps of the 2^16-mode gradient workload, "
                         "then 20 of a batch of 32 such fields")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this implementation runs on one GPU; --gpus must be 1 "
              "(the multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

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
        # the same 20 reverse long steps for a batch of 32 such fields
        import numpy as np
        sig = np.random.default_rng(7).uniform(0.8, 1.2, 32).tolist()
        bp = P.MPABatchPlan([g.grid.n] * 32, g.grid.dt, g.dmmap, gs.L, gs.M, gs.n_iter, gs.block, gs.halo,
                            P.MPA_C64, gs.omega_band, sigma_scale=sig)
        xb = torch.from_numpy(np.concatenate([g.field(seed=g.seed + i) for i in range(32)])).to(
            device="cuda:0", dtype=torch.complex64)
        ck = bp.propagate_checkpointed(xb, 0.0, 20 * gs.L)
        bp.adjoint(ck, (2 * xb).contiguous(), 0.0, 20 * gs.L)
        torch.cuda.synchronize()
        bp.close()
        print(json.dumps({"pmc_grad": True, "reverse_launches": 20, "batch_reverse_launches": 20}), flush=True)
        return

    if args.profile_large:
        # blocks above 4096 (four-step windows, node order) at the headline's dz
        w = WORKLOADS[HEADLINE]
        dz = w.mpa.L / w.mpa.M
        x = torch.from_numpy(w.field()).to(device="cuda:0", dtype=torch.complex64)
        for block, halo, M, shift in ((8192, 1024, 4, 192), (16384, 4096, 16, 769)):
            pl = P.MPAPlan(w.grid.n, w.grid.dt, w.dmmap, M * dz, M, w.mpa.n_iter, block, halo, P.MPA_C64,
                           w.mpa.omega_band, shift=shift)
            pl.propagate(x, 0.0, 10 * M * dz)
            torch.cuda.synchronize()
            pl.close()
        print(json.dumps({"profile_large": True, "long_steps_each": 10}), flush=True)
        return

    w = WORKLOADS[HEADLINE]
    s = w.mpa
    n = w.grid.n
    launches_per_step = int(round(STEP_Z / s.L))
    log(f"workload {w.name}: N={n} B={s.block} H={s.halo} shift={s.shift} L={s.L} M={s.M} n_iter={s.n_iter}")
    a0 = w.field()
    plan = _plan(P, w)
    info = plan.info()
    x = torch.from_numpy(a0).to(device="cuda:0", dtype=torch.complex64)

    if args.pmc_pass or args.profile_pass:
        if args.pmc_pass:
            # counter calibration: one copy of 512 MiB whose source was written
            # first in a 2 GiB fill, so that the 256 MiB last-level cache no
            # longer holds it (a copy of a cache-resident source fetches nothing)
            src = torch.ones(1 << 28, dtype=torch.complex64, device="cuda:0")      # 2 GiB
            dst = torch.empty(1 << 26, dtype=torch.complex64, device="cuda:0")     # 512 MiB
            torch.cuda.synchronize()
            dst.copy_(src[: 1 << 26])        # one copy kernel: reads 512 MiB, writes 512 MiB
            torch.cuda.synchronize()
            del src, dst
        plan.propagate(x, 0.0, (20 if args.pmc_pass else 40) * s.L)
        torch.cuda.synchronize()
        if args.profile_pass:
            dz = s.L / s.M
            for prec in (P.MPA_C64, P.MPA_C128):
                ss = P.SSPlan(n, w.grid.dt, w.dmmap, dz, prec)
                y = torch.from_numpy(a0).to(device="cuda:0", dtype=torch.complex64 if prec == 0 else torch.complex128)
                ss.propagate(y, 0.0, 20 * dz)
                torch.cuda.synchronize()
                ss.close()
        plan.close()
        print(json.dumps({"pmc_pass" if args.pmc_pass else "profile_pass": True, "copy_bytes": 1 << 29}),
              flush=True)
        return

    z = 0.0
    for _ in range(args.warmup):
        plan.propagate(x, z, z + STEP_Z)
        z += STEP_Z
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        plan.propagate(x, z, z + STEP_Z)
        z += STEP_Z
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    mode_steps = n * s.M * launches_per_step * args.steps
    value = mode_steps / wall
    launch_s = gpu_ms * 1e-3 / (launches_per_step * args.steps)
    fl = flops_per_block(info["block"], s.M, s.n_iter) * info["n_blocks"]
    achieved = fl / launch_s / 1e12
    eff_gbps = value * 32.0 * s.n_iter / 1e9
    cfg = f"B={s.block} H={s.halo} shift={s.shift} L={s.L:g} M={s.M} n_iter={s.n_iter}"
    traffic = measured_traffic(cfg)
    log(f"MPA: {value:.3e} mode-steps/s, {launch_s * 1e6:.2f} us per long-step launch, "
        f"{achieved:.2f} TFLOP/s algorithmic, effective {eff_gbps:.0f} GB/s")
    out = {
        "metric": "mode-steps/s, MPA vs split-step, 1 MI355X, at stated rel-L2 error vs FP64",
        "value": value, "unit": "mode-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "n_modes": n, "channels": w.n_channels,
                   "modulation": w.modulation, "block": info["block"], "halo": info["halo"],
                   "shift": info["shift"], "n_blocks": info["n_blocks"], "L": s.L, "M": s.M, "dz": s.L / s.M,
                   "n_iter": s.n_iter,
                   "step": f"z -> z + {STEP_Z:g} = {launches_per_step} long steps",
                   "precision": "FP32 node work, FP64 phases and carry"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": traffic,
                     "kernel": "mpa_block_kernel", "launch_us": launch_s * 1e6, "launch_config": cfg,
                     "flops_per_launch": fl,
                     "effective_GBps": eff_gbps, "effective_frac_of_hbm": eff_gbps / HBM_PEAK_GBPS,
                     "effective_convention": "32 B per mode per node evaluation (one read and one write of "
                                             "the FP32 complex field per transform pair), n_iter evaluations "
                                             "per dz",
                     "physical_GBps": (traffic / launch_s / 1e9) if traffic else None},
    }
    plan.close()

    if not args.no_compare:
        out.update(compare(w, a0, torch, P, value))
    if not args.no_extra:
        out["dm1ch_n4096_f64"] = c1_section(torch, P)
        out["wdm8_n262144"] = c2_section(torch, P)
        out["batched"] = batched(torch, P)
        out["autotune_wdm32"] = autotune_table(WORKLOADS[HEADLINE], torch, P, launches=20)
        out["gradient"] = gradient(torch, P, args.grad_periods)
        out["batched_gradient"] = batched_gradient(torch, P)
    if not args.no_cpu:
        log("CPU oracle baselines ...")
        out["cpu_baseline"] = cpu_baseline(w)
        out["cpu_baseline_all_cores"] = cpu_all_cores(w)
    out["paper_context"] = paper_context()
    print(json.dumps(out), flush=True)


def paper_context():
    """The paper's own CPU numbers, with its hardware (context only, another
    machine and workload): read from the numbers the test suite pins."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "paper_numbers.json")
    with open(path) as f:
        g = json.load(f)
    keys = ("cpu_speedup_over_one_processor", "near_linear_scaling_up_to_processors",
            "ss_over_mpa_time_ratio_32_cores_n2")
    return {"note": "the paper's shared-memory CPU runs: another machine and workload, not a target",
            **{k: g[k] for k in keys if k in g}}


# ---- accuracy and the split-step comparator -----------------------------------------

def _interp_time(points, err):
    """Time at error `err` by log-log interpolation between the two sweep
    points (error, seconds) that bracket it; None when none do."""
    pts = sorted(points)
    for (e0, t0), (e1, t1) in zip(pts, pts[1:]):
        if e0 <= err <= e1 and e0 > 0 and e1 > e0:
            f = (math.log(err) - math.log(e0)) / (math.log(e1) - math.log(e0))
            return math.exp(math.log(t0) + f * (math.log(t1) - math.log(t0)))
    return None


def compare(w, a0, torch, P, value):
    """After z = ACC_Z: MPA (stated configuration, 2 and 1 sweeps; and the
    same method in one full window, which gives the blocking error at full
    size) and split-step (both precisions, dz swept) against an FP64 split-step
    reference at dz/32 (its distance to the dz/16 run is reported), relative
    L2 over the full band and over the channels' band |omega| <= band + 50
    (the blocked roll-off removes only out-of-band four-wave-mixing products,
    which the grid aliases); then the split-step time at the MPA's error, by
    interpolation along each precision's sweep, and the ratio to the MPA's."""
    import numpy as np
    s = w.mpa
    n, dt = w.grid.n, w.grid.dt
    dz = s.L / s.M

    def run_ss(h, prec, reps=1):
        pl = P.SSPlan(n, dt, w.dmmap, h, prec)
        cdt = torch.complex64 if prec == P.MPA_C64 else torch.complex128
        el = None
        for _ in range(reps):
            y = torch.from_numpy(a0).to(device="cuda:0", dtype=cdt)
            el, _ = _timed(torch, lambda: pl.propagate(y, 0.0, ACC_Z))
        pl.close()
        return y.cpu().numpy().astype(np.complex128), el

    log("FP64 split-step reference ...")
    r16, _ = run_ss(dz / 16, P.MPA_C128)
    ref, _ = run_ss(dz / 32, P.MPA_C128)
    omega = 2 * math.pi * np.fft.fftfreq(n, dt)
    band = np.abs(omega) <= s.omega_band + 50.0
    ref_band = np.fft.ifft(ref)[band]

    def err(a):
        full = float(np.linalg.norm(a - ref) / np.linalg.norm(ref))
        inb = float(np.linalg.norm(np.fft.ifft(a)[band] - ref_band) / np.linalg.norm(ref_band))
        return full, inb

    ref_full, ref_in = err(r16)
    del r16
    mpa = []
    blocked = None
    for nit in (s.n_iter, 1):
        pl = _plan(P, w, n_iter=nit)
        y = torch.from_numpy(a0).to(device="cuda:0", dtype=torch.complex64)
        pl.propagate(y, 0.0, 8 * s.L)
        y = torch.from_numpy(a0).to(device="cuda:0", dtype=torch.complex64)
        el, _ = _timed(torch, lambda: pl.propagate(y, 0.0, ACC_Z))
        pl.close()
        out = y.cpu().numpy().astype(np.complex128)
        if blocked is None:
            blocked = out
        e_full, e_in = err(out)
        mpa.append({"n_iter": nit, "rel_l2_in_band": e_in, "rel_l2_full_band": e_full, "seconds": el,
                    "mode_steps_per_s": n * ACC_Z / dz / el})
        log(f"MPA n_iter={nit}: in-band {e_in:.3e} full-band {e_full:.3e}, {el * 1e3:.0f} ms")
    # the blocking error at full size: the same method and precision without time blocks
    pw = P.MPAPlan(n, dt, w.dmmap, s.L, s.M, s.n_iter, 0, 0, P.MPA_C64, s.omega_band)
    y = torch.from_numpy(a0).to(device="cuda:0", dtype=torch.complex64)
    el_w, _ = _timed(torch, lambda: pw.propagate(y, 0.0, ACC_Z))
    pw.close()
    whole = y.cpu().numpy().astype(np.complex128)
    e_full_w, e_in_w = err(whole)
    fb, fw = np.fft.ifft(blocked), np.fft.ifft(whole)
    blocking = {"full_window_rel_l2_in_band": e_in_w, "full_window_rel_l2_full_band": e_full_w,
                "full_window_seconds": el_w,
                "blocked_vs_full_window_in_band": float(np.linalg.norm((fb - fw)[band]) / np.linalg.norm(fw[band])),
                "blocked_vs_full_window_full_band": float(np.linalg.norm(blocked - whole) / np.linalg.norm(whole))}
    del fb, fw, whole, blocked
    log(f"full window (no blocks): in-band {e_in_w:.3e} full-band {e_full_w:.3e}, {el_w * 1e3:.0f} ms; "
        f"blocked vs full window {blocking['blocked_vs_full_window_in_band']:.2e} in band, "
        f"{blocking['blocked_vs_full_window_full_band']:.2e} full band")
    sweep = []
    for k in (0.5, 1.0, 2.0, 4.0):
        h = dz / k
        for prec, label in ((P.MPA_C64, "f32"), (P.MPA_C128, "f64")):
            a, el = run_ss(h, prec, reps=2)
            e_full, e_in = err(a)
            sweep.append({"dz": h, "precision": label, "rel_l2_in_band": e_in, "rel_l2_full_band": e_full,
                          "seconds": el, "mode_steps_per_s": n * ACC_Z / h / el})
            log(f"SS {label} dz={h:.3e}: in-band {e_in:.3e} full-band {e_full:.3e}, {el * 1e3:.0f} ms")
    eq = {}
    e_mpa, t_mpa = mpa[0]["rel_l2_in_band"], mpa[0]["seconds"]
    for label in ("f32", "f64"):
        pts = [(r["rel_l2_in_band"], r["seconds"]) for r in sweep if r["precision"] == label]
        t = _interp_time(pts, e_mpa)
        dz_eq = None
        pd = sorted((r["rel_l2_in_band"], r["dz"]) for r in sweep if r["precision"] == label)
        for (e0, h0), (e1, h1) in zip(pd, pd[1:]):
            if e0 <= e_mpa <= e1:
                f = (math.log(e_mpa) - math.log(e0)) / (math.log(e1) - math.log(e0))
                dz_eq = math.exp(math.log(h0) + f * (math.log(h1) - math.log(h0)))
        eq[label] = {"seconds_at_mpa_error": t, "time_ratio_ss_over_mpa": (t / t_mpa) if t else None,
                     "dz_at_mpa_error": dz_eq, "ss_dz_over_mpa_dz": (dz_eq / dz) if dz_eq else None}
        log(f"equal accuracy ({e_mpa:.3e}), split-step {label}: "
            + (f"{t * 1e3:.0f} ms, ratio {t / t_mpa:.2f}" if t else "not bracketed"))
    return {"accuracy": {"z": ACC_Z, "mpa_rel_l2_in_band": e_mpa, "mpa_rel_l2_full_band": mpa[0]["rel_l2_full_band"],
                         "in_band": f"|omega| <= {s.omega_band + 50.0:g}",
                         "reference": f"FP64 split-step on the GPU at dz = {dz / 32:.4e}; the dz/16 run differs from it "
                                      f"by {ref_in:.1e} in band, {ref_full:.1e} full band",
                         "mpa": mpa, "blocking_error": blocking},
            "split_step": {"sweep": sweep, "equal_accuracy": eq}}


# ---- the 8-channel 2^18-mode workload ---------------------------------------------

def c2_section(torch, P):
    """The 8-channel OOK workload (2^18 modes): throughput of the stated
    configuration (4096-blocks, 512-halos, L = 2.5e-4, M = 4) and of the
    autotuner's pick at the same dz, with the in-band error after one period
    against an FP64 split-step at dz = 3.9e-6 (its distance to dz = 7.8e-6
    reported), and the split-step FP32 time at the same error."""
    import numpy as np
    from paper_1101_0086_amd.autotune import autotune
    from workloads import WORKLOADS
    w = WORKLOADS["wdm8_n262144_f32"]
    s = w.mpa
    n, dt = w.grid.n, w.grid.dt
    a0 = w.field()

    def run_ss(h, prec):
        pl = P.SSPlan(n, dt, w.dmmap, h, prec)
        y = torch.from_numpy(a0).to(device="cuda:0", dtype=torch.complex64 if prec == 0 else torch.complex128)
        el, _ = _timed(torch, lambda: pl.propagate(y, 0.0, 1.0))
        pl.close()
        return y.cpu().numpy().astype(np.complex128), el

    r1, _ = run_ss(0.5 / 64000, P.MPA_C128)
    ref, _ = run_ss(0.5 / 128000, P.MPA_C128)
    omega = 2 * math.pi * np.fft.fftfreq(n, dt)
    band = np.abs(omega) <= s.omega_band + 50.0
    rb = np.fft.ifft(ref)[band]

    def err(a):
        return float(np.linalg.norm(np.fft.ifft(a)[band] - rb) / np.linalg.norm(rb))

    rows = {}
    dzq = s.L / s.M
    pick, _ = autotune(torch.from_numpy(a0).to(device="cuda:0", dtype=torch.complex64), dt, w.dmmap, dzq, s.n_iter,
                       s.omega_band, launches=20)
    for name, kw in (("stated", {}), ("autotuned", dict(block=pick.block, halo=pick.halo, L=pick.L, M=pick.M,
                                                          shift=pick.shift))):
        pl = _plan(P, w, **kw)
        y = torch.from_numpy(a0).to(device="cuda:0", dtype=torch.complex64)
        pl.propagate(y, 0.0, 0.02)
        y = torch.from_numpy(a0).to(device="cuda:0", dtype=torch.complex64)
        el, _ = _timed(torch, lambda: pl.propagate(y, 0.0, 1.0))
        pl.close()
        rows[name] = {**({"block": s.block, "halo": s.halo, "L": s.L, "M": s.M, "shift": s.shift} if not kw else kw),
                      "rel_l2_in_band_one_period": err(y.cpu().numpy().astype(np.complex128)),
                      "seconds_one_period": el, "mode_steps_per_s": n / dzq / el}
        log(f"2^18 {name}: {rows[name]['mode_steps_per_s']:.3e} mode-steps/s, in-band "
            f"{rows[name]['rel_l2_in_band_one_period']:.3e}")
    ss = {}
    for prec, label in ((P.MPA_C64, "f32"), (P.MPA_C128, "f64")):
        a, el = run_ss(dzq, prec)
        a, el = run_ss(dzq, prec)
        ss[label] = {"dz": dzq, "rel_l2_in_band_one_period": err(a), "seconds_one_period": el,
                     "mode_steps_per_s": n / dzq / el}
    return {"workload": w.name, "mpa": rows, "split_step_same_dz": ss,
            "reference": "FP64 split-step at dz = 3.9e-6; dz = 7.8e-6 differs from it by "
                         f"{err(r1):.1e} in band"}


def c1_section(torch, P):
    """The single-channel FP64 workload (2^12 modes, one window, L = 0.05,
    M = 16, n_iter = 3) over its 10 map periods: MPA time and error, in the
    fused (wavefront) schedule and in the paper's node-parallel schedule (the
    sixteen nodes of a sweep in workgroups of their own: one window leaves
    the fused kernel a single workgroup), against an FP64 split-step at dz/64
    (its distance to dz/128 reported), the FP64 split-step swept over 4, 2, 1
    and 1/2 times the MPA's dz, and its time at the MPA's error by
    interpolation."""
    import numpy as np
    from workloads import WORKLOADS
    w = WORKLOADS["dm1ch_n4096_f64"]
    s = w.mpa
    n, dt = w.grid.n, w.grid.dt
    z1 = float(w.periods)
    dz = s.L / s.M
    a0 = w.field()

    def run_ss(h):
        pl = P.SSPlan(n, dt, w.dmmap, h, P.MPA_C128)
        y = torch.from_numpy(a0).to(device="cuda:0", dtype=torch.complex128)
        pl.propagate(y, 0.0, 2 * s.L)                 # warm-up
        y = torch.from_numpy(a0).to(device="cuda:0", dtype=torch.complex128)
        el, _ = _timed(torch, lambda: pl.propagate(y, 0.0, z1))
        pl.close()
        return y.cpu().numpy(), el

    r128, _ = run_ss(dz / 128)
    ref, _ = run_ss(dz / 64)

    def err(a):
        return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))

    mpa = {}
    for name, sched in (("wavefront", P.MPA_WAVEFRONT), ("node_parallel", P.MPA_NODE_PARALLEL)):
        pl = P.MPAPlan(n, w.grid.dt, w.dmmap, s.L, s.M, s.n_iter, 0, 0, P.MPA_C128, s.omega_band, schedule=sched)
        y = torch.from_numpy(a0).to(device="cuda:0", dtype=torch.complex128)
        pl.propagate(y, 0.0, 2 * s.L)
        y = torch.from_numpy(a0).to(device="cuda:0", dtype=torch.complex128)
        el, _ = _timed(torch, lambda: pl.propagate(y, 0.0, z1))
        pl.close()
        mpa[name] = {"rel_l2": err(y.cpu().numpy()), "seconds": el, "mode_steps_per_s": n * z1 / dz / el}
    sweep = []
    for k in (0.25, 0.5, 1, 2):             # dz 4, 2, 1 and 1/2 times the MPA's
        a, t = run_ss(dz / k)
        sweep.append({"dz": dz / k, "rel_l2": err(a), "seconds": t, "mode_steps_per_s": n * z1 * k / dz / t})
    for name, r in mpa.items():
        t_ss = _interp_time([(q["rel_l2"], q["seconds"]) for q in sweep], r["rel_l2"])
        r["split_step_seconds_at_mpa_error"] = t_ss
        r["time_ratio_ss_over_mpa"] = (t_ss / r["seconds"]) if t_ss else None
        log(f"2^12 FP64 MPA ({name}): {r['mode_steps_per_s']:.3e} mode-steps/s at {r['rel_l2']:.3e}, "
            f"split-step / MPA time at that error {r['time_ratio_ss_over_mpa']}")
    return {"workload": w.name, "precision": "FP64", "distance": z1, "L": s.L, "M": s.M, "n_iter": s.n_iter,
            "mpa": mpa, "split_step_f64": sweep,
            "reference": f"FP64 split-step at dz/64; the dz/128 run differs from it by {err(r128):.1e}"}


# ---- batches, autotuner, gradients ---------------------------------------------------

def batched(torch, P, count=256, steps=200):
    """256 independent fields, N uniform over 2^14..2^18, 1-16 channels,
    sigma uniform in [0.5, 2], 4096-blocks with 512-halos, L = 5e-5, M = 1,
    2 sweeps: one launch per long step for all instances, eager and as a
    replayed HIP graph of `steps` long steps; and the autotuner's candidates
    for the shortest instance at the same dz (blocks of at most 4096, the
    batch kernel's)."""
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
    t_eager, _ = _timed(torch, lambda: bp.propagate(x, 0.0, z1))
    g = bp.capture(x, 0.0, z1)
    g.launch()
    t_graph, _ = _timed(torch, lambda: g.launch())
    g.close()
    bp.close()
    ms = info["total_samples"] * M * steps
    log(f"batched: {info['work_items']} work items, eager {ms / t_eager:.3e}, graph {ms / t_graph:.3e} mode-steps/s")
    from paper_1101_0086_amd.autotune import candidates
    dz = L / M
    tuned = []
    for c in candidates(min(ns), dt, dm_map(beta3=0.1), dz, band, blocks=(512, 1024, 2048, 4096)):
        cp = P.MPABatchPlan(ns, dt, dm_map(beta3=0.1), c.L, c.M, nit, c.block, c.halo, P.MPA_C64, band,
                            sigma_scale=sig, shift=c.shift)
        y = x.clone()
        cp.propagate(y, 0.0, 4 * c.L)
        el, _ = _timed(torch, lambda: cp.propagate(y, 0.0, z1))
        cp.close()
        tuned.append({"block": c.block, "halo": c.halo, "shift": c.shift, "L": c.L, "M": c.M,
                      "mode_steps_per_s": info["total_samples"] * (z1 / dz) / el})
    best = max(tuned, key=lambda t: t["mode_steps_per_s"])
    log(f"batched autotune best: B={best['block']} H={best['halo']} shift={best['shift']} M={best['M']}: "
        f"{best['mode_steps_per_s']:.3e}")
    return {"instances": count, "total_modes": info["total_samples"], "work_items_per_launch": info["work_items"],
            "L": L, "M": M, "n_iter": nit, "block": 4096, "halo": 512, "long_steps": steps,
            "mode_steps_per_s_eager": ms / t_eager, "mode_steps_per_s_graph": ms / t_graph,
            "us_per_long_step_graph": t_graph / steps * 1e6, "block_overlap_shift_at_same_dz": tuned}


def autotune_table(w, torch, P, launches=20):
    """Autotuner over (block, halo, L, M, shift) at the workload's dz."""
    from paper_1101_0086_amd.autotune import autotune
    s = w.mpa
    x = torch.from_numpy(w.field()).to(device="cuda:0", dtype=torch.complex64)
    dz = s.L / s.M
    rows = []
    for shifted in (True, False):
        best, cands = autotune(x, w.grid.dt, w.dmmap, dz, s.n_iter, s.omega_band, launches=launches,
                               shifted=shifted)
        rows += [{"block": c.block, "halo": c.halo, "shift": c.shift, "L": c.L, "M": c.M,
                  "mode_steps_per_s": w.grid.n / (c.seconds_per_unit_z * dz)} for c in cands]
        log(f"autotune {w.name} ({'shifted' if shifted else 'unshifted'}): best B={best.block} H={best.halo} "
            f"shift={best.shift} M={best.M}: {w.grid.n / (best.seconds_per_unit_z * dz):.3e}")
    return {"dz": dz, "candidates": rows}


def adjoint_flops_per_block(B: int, M: int, n_iter: int) -> float:
    """Algorithmic flops of the reverse pass of one block and long step:
    4 n_iter M + 7 transforms (recomputed forward and reverse) of 5 B log2 B
    flops, and about 100 n_iter M + 60 flops per point of elementwise work."""
    return 5.0 * B * math.log2(B) * (4 * n_iter * M + 7) + B * (100.0 * n_iter * M + 60)


def gradient(torch, P, periods=20):
    """Gradient workload: 2^16 modes, 4 OOK channels, `periods` map periods
    (B = 2048, H = 256, L = 2.5e-4, M = 2, 2 sweeps, FP32 node work), loss =
    sum |A(z1) - target|^2: the plain forward, the checkpointed forward (one
    checkpoint per period) and the reverse pass (each period recomputed from
    its checkpoint, the next period's recompute overlapped with the current
    period's reverse launches), timed separately after a warm-up."""
    from workloads import WORKLOADS
    w = WORKLOADS["wdm4_n65536_f32"]
    s = w.mpa
    a = w.field()
    plan = _plan(P, w)
    x0 = torch.from_numpy(a).to(device="cuda:0", dtype=torch.complex64)
    target = torch.from_numpy(w.field(seed=w.seed + 100)).to(device="cuda:0", dtype=torch.complex64)
    z1 = float(periods)
    steps = int(round(z1 / s.L))
    x = x0.clone()
    ck = plan.propagate_checkpointed(x, 0.0, 20 * s.L)            # warm-up, workspace
    plan.adjoint(ck, (2 * x).contiguous(), 0.0, 20 * s.L)
    x = x0.clone()
    t_fwd, _ = _timed(torch, lambda: plan.propagate(x, 0.0, z1))
    x = x0.clone()
    t_ck, ck = _timed(torch, lambda: plan.propagate_checkpointed(x, 0.0, z1))
    g = (2 * (x - target)).contiguous()
    t_adj, pg = _timed(torch, lambda: plan.adjoint(ck, g, 0.0, z1))
    kept = _kept_inputs(torch, plan, x0, z1, steps, lambda y: (2 * (y - target)).contiguous())
    nb = plan.info()["n_blocks"]
    plan.close()
    fl = adjoint_flops_per_block(s.block, s.M, s.n_iter) * nb
    r = {"workload": w.name, "n_modes": w.grid.n, "periods": periods, "long_steps": steps, "block": s.block,
         "halo": s.halo, "L": s.L, "M": s.M, "n_iter": s.n_iter, "n_blocks": nb, "checkpoints": int(ck.shape[0]),
         "forward_s": t_fwd, "checkpointed_forward_s": t_ck, "reverse_s": t_adj,
         "gradient_over_forward": (t_ck + t_adj) / t_fwd,
         "gradient_mode_steps_per_s": w.grid.n * s.M * steps / (t_ck + t_adj),
         "reverse_us_per_long_step": t_adj / steps * 1e6,
         "adjoint_flops_per_launch": fl,
         "adjoint_tflops_wall": fl * steps / t_adj / 1e12,
         "kept_inputs": dict(kept, gradient_over_forward=(kept["checkpointed_forward_s"] + kept["reverse_s"]) / t_fwd)}
    log(f"gradient ({periods} periods): forward {t_fwd:.2f} s, checkpointed {t_ck:.2f} s, reverse {t_adj:.2f} s "
        f"({r['gradient_over_forward']:.2f}x forward; step inputs kept: "
        f"{r['kept_inputs']['gradient_over_forward']:.2f}x)")
    return r


# HBM budget for the step inputs kept by the checkpointed forward (the
# gradient runs keep 40 GiB and 62.5 GiB of the MI355X's 288 GB)
KEEP_BYTES = 96 << 30


def _kept_inputs(torch, plan, x0, z1, steps, grad_of):
    """The same checkpointed forward and reverse pass with every step input
    kept by the forward (plan.keep_inputs): one untimed run sizes the
    workspace, then both are timed."""
    plan.keep_inputs(KEEP_BYTES)
    x = x0.clone()
    ck = plan.propagate_checkpointed(x, 0.0, z1)
    plan.adjoint(ck, grad_of(x), 0.0, z1)
    del ck
    x = x0.clone()
    t_ck, ck = _timed(torch, lambda: plan.propagate_checkpointed(x, 0.0, z1))
    g = grad_of(x)
    t_adj, _ = _timed(torch, lambda: plan.adjoint(ck, g, 0.0, z1))
    plan.keep_inputs(0)
    del ck
    return {"checkpointed_forward_s": t_ck, "reverse_s": t_adj, "kept_bytes": int(x0.numel() * x0.element_size() * steps)}


def batched_gradient(torch, P, count=32, periods=1):
    """Gradients of 32 instances of the 2^16-mode 4-channel workload (seeds
    differ, sigma scales uniform in [0.8, 1.2]) through one map period with
    one batched launch per long step: checkpointed forward and reverse pass
    against the plain batched forward."""
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
    x = x0.clone()
    ck = bp.propagate_checkpointed(x, 0.0, 20 * s.L)              # warm-up, workspace
    bp.adjoint(ck, (2 * x).contiguous(), 0.0, 20 * s.L)
    x = x0.clone()
    t_fwd, _ = _timed(torch, lambda: bp.propagate(x, 0.0, z1))
    x = x0.clone()
    t_ck, ck = _timed(torch, lambda: bp.propagate_checkpointed(x, 0.0, z1))
    g = (2 * x).contiguous()
    t_adj, _ = _timed(torch, lambda: bp.adjoint(ck, g, 0.0, z1))
    del ck
    kept = _kept_inputs(torch, bp, x0, z1, steps, lambda y: (2 * y).contiguous())
    bp.close()
    ms = info["total_samples"] * s.M * steps
    r = {"workload": f"{count} x {w.name}", "total_modes": info["total_samples"],
         "work_items_per_launch": info["work_items"], "long_steps": steps,
         "forward_s": t_fwd, "checkpointed_forward_s": t_ck, "reverse_s": t_adj,
         "gradient_over_forward": (t_ck + t_adj) / t_fwd,
         "forward_mode_steps_per_s": ms / t_fwd,
         "gradient_mode_steps_per_s": ms / (t_ck + t_adj),
         "reverse_us_per_long_step": t_adj / steps * 1e6,
         "kept_inputs": dict(kept, gradient_over_forward=(kept["checkpointed_forward_s"] + kept["reverse_s"]) / t_fwd,
                             gradient_mode_steps_per_s=ms / (kept["checkpointed_forward_s"] + kept["reverse_s"]))}
    log(f"batched gradient ({count} instances): gradient {r['gradient_over_forward']:.2f}x forward "
        f"(step inputs kept: {r['kept_inputs']['gradient_over_forward']:.2f}x)")
    return r


# ---- CPU baselines (the oracle on the host) ------------------------------------------

def cpu_baseline(w, budget_s: float = 10.0):
    """The FP64 oracle (blocked MPA, NumPy, one thread) on the headline
    workload: whole long steps of the oracle's own march (same partition,
    taper, roll-off and shift as the GPU) from the seeded field, until the
    budget is spent; mode-steps/s."""
    import oracle as O
    s = w.mpa
    n, dt = w.grid.n, w.grid.dt
    a = w.field()
    t0 = time.perf_counter()
    steps = 0
    while True:
        a = O.mpa_step(a, dt, w.dmmap, s.L, s.M, s.n_iter, steps, s.block, s.halo, s.shift)
        steps += 1
        el = time.perf_counter() - t0
        if el > budget_s or steps >= 50:
            break
    model, cores = host_cpu()
    return {"value": n * s.M * steps / el, "unit": "mode-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} long steps of the 2^22-mode workload (L = {s.L:g}, M = {s.M}, "
                      f"{-(-n // (s.block - 2 * s.halo))} blocks each), {el:.1f} s, NumPy FFT on one thread",
            "host_cpu": model, "host_cores": cores}


def cpu_all_cores(w, long_steps: int = 1):
    """The paper's own decomposition of a long step on every host core (a
    thread pool over the z-nodes of each sweep for steps 2-4, harmonic
    ranges for step 5), full window of the headline field, against the same
    code on one thread; mode-steps/s."""
    import numpy as np

    import oracle as O
    from oracle.parallel import mpa_long_step_parallel
    s = w.mpa
    n, dt = w.grid.n, w.grid.dt
    a = w.field()
    om = O.omega_grid(n, dt)
    model, cores = host_cpu()
    res = {}
    for workers in (cores, 1):
        t0 = time.perf_counter()
        y = a
        for _ in range(long_steps):
            y = mpa_long_step_parallel(y, om, w.dmmap.beta2[0], w.dmmap.beta3[0], w.dmmap.sigma[0], w.dmmap.gamma,
                                       s.L, s.M, s.n_iter, workers=workers)
        res[workers] = time.perf_counter() - t0
    return {"value": n * s.M * long_steps / res[cores], "unit": "mode-steps/s", "cores": cores,
            "kind": "oracle, the paper's node-parallel decomposition",
            "sample": f"{long_steps} full-window long step(s) of the 2^22-mode field (L = {s.L:g}, M = {s.M}, "
                      f"{s.n_iter} sweeps), {res[cores]:.1f} s on {cores} threads, {res[1]:.1f} s on one",
            "one_thread_value": n * s.M * long_steps / res[1], "speed_up": res[1] / res[cores],
            "host_cpu": model}


if __name__ == "__main__":
    main()
