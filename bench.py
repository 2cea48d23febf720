#!/usr/bin/env python3
"""Benchmark of the structure-preserving FDTD reduction hot path on one MI355X.

Workload (3-D lossy PEC cavity, 128^3 cells of 1 mm; eps_r ~ U[1,4] and
sigma_e ~ U[0, 0.01] S/m constant on 8^3-cell blocks, seed 1; 4 z-directed
point ports driven together with seeded +-1 signs, sine-modulated Gaussian
f0 = 1.5 GHz, bandwidth 1.5 GHz).  One benchmark step is one pass of the whole
hot path:
  1. full-order leapfrog, 4000 steps at 0.99 x CFL, FP32 fields   (fdtd_step)
  2. SPRIM reduction, q = 200, 5 expansion points (M = 1.1,
     f_max = 3 GHz), FP32 complex COCG solves to 1e-4, FP64 CGS2 / CholQR2
     and FP64 projection                                           (mor_reduce)
  3. singular-value clamp at s = 4.95 (5 x the full step), FP64   (rom_perturb)
  4. reduced leapfrog, 800 steps at s = 4.95, FP32 state           (rom_step)
Metric: Gcell-updates/s = (cells x leapfrog steps + cells x Schur matvecs
(one per active column per COCG iteration; a column stops when it has
converged)) / time per step.  Outside the timed
region the script measures the end-to-end speedup against plain FP64
full-order FDTD (4000 steps at s = 0.99) at <= 1e-3 probe error, the live
per-kernel durations (HIP events on the launch stream) for the roofline, and
the CPU oracle on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the dominant kernels, from two rocprofv3 --pmc runs
# of `bench.py --counters --q 40` (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch averaged over the run's dispatches, same launch configuration as
# the timed step; the passes that update x and those that skip it alternate,
# so the figures average the two kernel variants).  A 1 GiB device copy in the
# same runs reads 524,311 KiB and writes 1,048,576 KiB, so FETCH is scaled by
# 2.0 and WRITE by 1.0.  A COCG
# pass skips converged columns, so each figure is kept with the algorithmic
# bytes per launch of that run (3.61 active columns of 4 per pass) and scaled
# to the active columns of the run that reports it.  The figures belong to the
# kernel source they were taken on: on any change to that file the traffic is
# reported null.
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
KERNEL_TRAFFIC = {
    "cocg_fused": {"src": "paper_1406_7042_amd/csrc/krylov.hip", "sha256_16": "78512adcc88a3b62",
                   "fetch_kib": 465149.0, "write_kib": 641027.3,
                   "alg_bytes_per_launch": 1420047845.1},
    "cocg_fused_real": {"src": "paper_1406_7042_amd/csrc/krylov.hip", "sha256_16": "78512adcc88a3b62",
                        "fetch_kib": 220664.6, "write_kib": 321845.1,
                        "alg_bytes_per_launch": 713169650.5},
    # the one-pass COCG pass of the 256^3 cavity's 16-column sweep
    # (`bench.py --workload cavity256` under the two counters)
    "cocg_fused_256": {"src": "paper_1406_7042_amd/csrc/krylov.hip", "sha256_16": "78512adcc88a3b62",
                       "fetch_kib": 14862073.6, "write_kib": 18478904.6,
                       "alg_bytes_per_launch": 39639767917.7},
    # one-pass leapfrog step on the 256^3 cavity (32-bit material numbers;
    # `bench.py --counters --n 256 --q 0`); these two serve the cavity256 workload only
    "fdtd_fused_256": {"src": "paper_1406_7042_amd/csrc/leapfrog_fused.hip", "sha256_16": "c50aed98e089f094",
                       "fetch_kib": 304923.6, "write_kib": 398334.4,
                       "alg_bytes_per_launch": 805306368.0},
}


def measured_traffic(name, per_launch_bytes=None):
    """HBM bytes per launch of `name` from the counter runs; scaled by the
    ratio of algorithmic bytes per launch (this run / the counter run) when
    given, since a COCG pass skips the columns that have converged and the
    two runs average over different mixes."""
    import hashlib
    t = KERNEL_TRAFFIC.get(name)
    if t is None:
        return None
    with open(os.path.join(ROOT, t["src"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != t["sha256_16"]:
            return None
    b = 1024 * (FETCH_SCALE * t["fetch_kib"] + WRITE_SCALE * t["write_kib"])
    if per_launch_bytes is not None and t.get("alg_bytes_per_launch"):
        b *= per_launch_bytes / t["alg_bytes_per_launch"]
    return int(b)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=128, help="cells per axis")
    p.add_argument("--q", type=int, default=200)
    p.add_argument("--full-steps", type=int, default=4000)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-accuracy", action="store_true")
    p.add_argument("--workload", choices=["cavity3d", "rom_batch", "board", "cavity256", "adjoint",
                                          "iris"],
                   default="cavity3d",
                   help="cavity3d: the benchmark step on the 128^3 cavity (default); "
                        "rom_batch: 256 reduced models from 96x96 cavities stepped 1e5 "
                        "steps beyond the CFL limit in one launch; board: the 256x128x64 "
                        "graded-mesh board reduced at q=300 and stepped at 9.9x the fine-cell "
                        "CFL step, with the reduced adjoint checked by central differences; "
                        "cavity256: FP32 leapfrog and a 16-RHS block Krylov sweep on a 256^3 "
                        "cavity (state far larger than the Infinity Cache); adjoint: probe-energy "
                        "gradients w.r.t. per-cell eps_r and sigma_e on the 512^2 design region; "
                        "iris: the 41x401 waveguide filter of Sec. V-B, waveform and S21 error "
                        "of the reduced model by s at M=1.1 and M=1.02")
    p.add_argument("--models", type=int, default=256, help="rom_batch: number of models")
    p.add_argument("--rom-steps", type=int, default=100_000, help="rom_batch: steps")
    p.add_argument("--counters", action="store_true",
                   help="short run for hardware-counter profiling: a 1 GiB device copy "
                        "(calibration), 20 leapfrog steps and one reduction at --q (none with "
                        "--q 0), no timing")
    return p.parse_args()


def counters_run(a, P, W, wl, op, signs, dt, mor_kw):
    """Kernels of one short pass for `rocprofv3 --pmc`: the copy of a known byte
    count calibrates FETCH_SIZE / WRITE_SIZE against the kernels of the path."""
    import torch
    dev = torch.device("cuda:0")
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    f32 = op.new_fields(torch.float32)
    u = torch.tensor(W.drive(wl, dt, 20, signs), dtype=torch.float32, device=dev)
    y = torch.zeros((20, 4), dtype=torch.float32, device=dev)
    P.fdtd_step(op, dt, 20, f32, wl.sources, u, wl.probes, y)
    torch.cuda.synchronize()
    if a.q == 0:  # leapfrog only
        print(json.dumps({"mode": "counters", "copy_bytes": 2 * (1 << 30), "n": a.n,
                          "leapfrog_steps": 20}), flush=True)
        return
    rom = P.mor_reduce(op, wl.sources, wl.probes, a.q, **mor_kw)
    torch.cuda.synchronize()
    info = rom.info()
    print(json.dumps({"mode": "counters", "copy_bytes": 2 * (1 << 30), "q": a.q,
                      "cocg_iters": info["solve_iters"], "matvecs": info["matvecs"],
                      "active_cols_per_launch": info["matvecs"] / max(info["solve_iters"], 1)}),
          flush=True)


def copy_ceiling_gbs():
    """Bytes read plus written per second by a 1 GiB device-to-device copy
    (torch's copy_, the runtime's copy kernel), timed with events on the
    current stream: the measured ceiling the roofline fraction is also
    reported against."""
    import torch
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * (1 << 30) * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return round(gbs, 1)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": a.gpus}), flush=True)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1406_7042_amd as P
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.workload == "rom_batch":
        rom_batch(a, P, W)
        return
    if a.workload == "board":
        board(a, P, W)
        return
    if a.workload == "cavity256":
        cavity256(a, P, W)
        return
    if a.workload == "adjoint":
        adjoint_design(a, P, W)
        return
    if a.workload == "iris":
        iris(a, P, W)
        return
    n = a.n
    wl = W.cavity3d(n=n, d=1e-3, seed=1, block=8, nports=4, f0=1.5e9, bw=1.5e9)
    signs = W.port_signs(1, 4)
    ncells = n ** 3
    log(f"[bench] building operator {n}^3")
    op = P.Operator.from_workload(wl)
    dt = 0.99 * op.dt_max
    nfull = a.full_steps
    kfac = 5  # s = 0.99 * 5 = 4.95
    dt_rom = kfac * dt
    nrom = nfull // kfac
    fmax = wl.f0 + wl.bw  # 3 GHz
    q = a.q
    u_full = torch.tensor(W.drive(wl, dt, nfull, signs), dtype=torch.float32, device=dev)
    u_rom = torch.tensor(W.drive(wl, dt_rom, nrom, signs), dtype=torch.float32, device=dev)
    f32 = op.new_fields(torch.float32)
    y_full = torch.zeros((nfull, 4), dtype=torch.float32, device=dev)
    mor_kw = dict(dt_ref=dt, fmax=fmax, M=1.1, L=2, tol=1e-4, max_iter=4000, defl_tol=1e-6,
                  precision="f32")

    if a.counters:
        counters_run(a, P, W, wl, op, signs, dt, mor_kw)
        return
    phase = {"fdtd": 0.0, "reduce": 0.0, "perturb": 0.0, "rom_step": 0.0}

    def one_step():
        t = time.perf_counter()
        f32.zero_()
        P.fdtd_step(op, dt, nfull, f32, wl.sources, u_full, wl.probes, y_full)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rom = P.mor_reduce(op, wl.sources, wl.probes, q, **mor_kw)
        t2 = time.perf_counter()
        ncl = P.rom_perturb(rom, dt_rom, 0.9999, dtype="f32")
        t3 = time.perf_counter()
        y = P.rom_step([rom], dt_rom, nrom, [u_rom], dtype="f32")[0]
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        for k_, v_ in zip(phase, (t1 - t, t2 - t1, t3 - t2, t4 - t3)):
            phase[k_] += v_
        return rom, ncl, y

    for w in range(a.warmup):
        log(f"[bench] warmup {w + 1}/{a.warmup}")
        one_step()
        torch.cuda.synchronize()
    for k_ in phase:
        phase[k_] = 0.0
    # HIP events on the launch stream time the Krylov iterations inside the
    # timed region; the 20 us leapfrog launches run untimed there (an event pair
    # costs more host time than such a launch) and are timed in a separate pass
    P.yeerom.profile_reset()
    P.yeerom.profile_select(["cocg_fused", "cocg_fused_real", "schur_h", "schur_e", "cocg_update"])
    P.yeerom.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    matvecs = 0
    infos = []
    for s in range(a.steps):
        rom, ncl, y = one_step()
        info = rom.info()
        matvecs += info["matvecs"]
        infos.append(info)
        log(f"[bench] step {s + 1}/{a.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    P.yeerom.profile_enable(False)
    T = (t1 - t0) / a.steps
    kernels = {}
    for name in ("cocg_fused", "cocg_fused_real", "schur_h", "schur_e", "cocg_update"):
        cnt, ms = P.yeerom.profile_read(name)
        kernels[name] = {"launches": cnt, "ms_total": ms, "us_avg": 1e3 * ms / max(cnt, 1)}
    # leapfrog half-step timings: 400 steps on their own, events on every launch
    P.yeerom.profile_reset()
    P.yeerom.profile_select(["fdtd_e", "fdtd_h", "fdtd_fused"])
    P.yeerom.profile_enable(True)
    f32.zero_()
    P.fdtd_step(op, dt, 400, f32, wl.sources, u_full[:400], wl.probes, y_full[:400])
    torch.cuda.synchronize()
    P.yeerom.profile_enable(False)
    P.yeerom.profile_select(None)
    for name in ("fdtd_e", "fdtd_h", "fdtd_fused"):
        cnt, ms = P.yeerom.profile_read(name)
        kernels[name] = {"launches": cnt, "ms_total": ms, "us_avg": 1e3 * ms / max(cnt, 1)}
    cell_updates = ncells * nfull + ncells * (matvecs / a.steps)
    value = cell_updates / T / 1e9

    # ---- roofline of the dominant kernel (algorithmic bytes per launch)
    # bytes per cell of what each step of the algorithm has to move, FP32:
    #   leapfrog half step: read E and H, write one of them: 9 values = 36 B
    #   Schur matvec sweep 1 (h = a22^-1 cp(x)): read x, write h: 6 complex = 48 B / RHS
    #   Schur matvec sweep 2 (y = W(a11 x - z curl_d h)): read x, h, write y: 72 B / RHS
    #   COCG update (x += a p, r -= a q): read x r p q, write x r: 144 B / RHS
    #   one-pass COCG iteration (r, p updates and q = S p, H on chip; x every
    #     other pass from the last two p): read r q p, write r q p (144 B / RHS),
    #     on every other pass also read x and p_{i-2} and write x (216 B / RHS):
    #     180 B / RHS on average, plus a11 (24 B) and the mask (3 B) once per
    #     cell; at the real expansion point the same pass in real arithmetic:
    #     90 B / RHS + 15 B
    # columns a COCG pass actually updates (a column stops once converged),
    # averaged over the passes of the reduction
    nb = (matvecs / a.steps) / max(infos[-1]["solve_iters"], 1)
    per_launch = {"fdtd_e": 36.0 * ncells, "fdtd_h": 36.0 * ncells, "fdtd_fused": 48.0 * ncells,
                  "cocg_fused": (180.0 * nb + 27.0) * ncells,
                  "cocg_fused_real": (90.0 * nb + 15.0) * ncells,
                  "schur_h": 48.0 * ncells * nb, "schur_e": 72.0 * ncells * nb,
                  "cocg_update": 144.0 * ncells * nb}
    kernels = {k: v for k, v in kernels.items() if v["launches"] > 0}
    dom = max(kernels, key=lambda k: kernels[k]["ms_total"])
    dur = kernels[dom]["us_avg"] * 1e-6
    achieved = per_launch[dom] / dur / 1e9 if dur > 0 else 0.0
    traffic = measured_traffic(dom, per_launch[dom])
    copy_gbs = copy_ceiling_gbs()
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "bytes_per_launch": per_launch[dom],
                "us_per_launch": round(kernels[dom]["us_avg"], 2),
                "traffic_gbs": round(traffic / dur / 1e9, 1) if traffic and dur > 0 else None,
                "copy_ceiling_gbs": copy_gbs,
                "frac_of_copy": round(achieved / copy_gbs, 4) if copy_gbs else None}

    out = {
        "metric": "Gcell-updates/s (FDTD+Krylov) & end-to-end speedup vs plain FDTD at <=1e-3 err",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(T * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"3-D lossy PEC cavity {n}^3 cells 1 mm, eps_r~U[1,4] and "
                               f"sigma_e~U[0,0.01] S/m on 8^3 blocks, 4 point ports; "
                               f"{nfull} leapfrog steps at 0.99 CFL + SPRIM q={q} + clamp + "
                               f"{nrom} reduced steps at 4.95 CFL",
                   "cells": ncells, "q": q, "parallelism": "single GPU"},
        "breakdown": {
            "reduce_s": round(sum(i["seconds_solve"] + i["seconds_orth"] + i["seconds_project"]
                                  for i in infos) / len(infos), 4),
            "solve_s": round(sum(i["seconds_solve"] for i in infos) / len(infos), 4),
            "orth_s": round(sum(i["seconds_orth"] for i in infos) / len(infos), 4),
            "project_s": round(sum(i["seconds_project"] for i in infos) / len(infos), 4),
            # projection: FP64 GEMMs of eq. (R_and_Freduced) on MFMA (rocBLAS):
            # V1^T De V1, V1^T Dse V1, V2^T Dm V2 (Dsm~ is exactly 0: no magnetic
            # loss) and V1^T (K V2), 2 n q^2 flop each, against the 78.6 TFLOP/s
            # FP64 peak
            "project_fp64_tflops": round(2.0 * (3 * op.ne_slots + op.nh_slots) * op.len * q * q
                                         / (sum(i["seconds_project"] for i in infos) / len(infos))
                                         / 1e12, 2),
            "matvecs_per_step": matvecs / a.steps,
            "cocg_iters": infos[-1]["solve_iters"],
            "relres_max": infos[-1]["relres_max"],
            "q1": infos[-1]["q1"], "q2": infos[-1]["q2"], "n_clamped": infos[-1]["n_clamped"],
            "fdtd_gcells": None,
            "phase_s": {k_: round(v_ / a.steps, 4) for k_, v_ in phase.items()},
        },
        "kernels": kernels,
        "roofline": roofline,
    }
    # leapfrog steps of the timing pass: two half-step launches or one one-pass launch each
    nlf = kernels.get("fdtd_e", {}).get("launches", 0) or kernels.get("fdtd_fused", {}).get("launches", 0)
    if nlf:
        ms_lf = sum(kernels.get(k_, {}).get("ms_total", 0.0) for k_ in ("fdtd_e", "fdtd_h", "fdtd_fused"))
        out["breakdown"]["fdtd_gcells"] = round(ncells / (ms_lf / nlf * 1e-3) / 1e9, 2)

    # ---- accuracy and end-to-end speedup (outside the timed region)
    if not a.no_accuracy:
        log("[bench] accuracy sweep")
        out["e2e"] = accuracy(P, W, wl, op, signs, dt, nfull, q, mor_kw)

    # ---- CPU oracle on a bounded sample
    if not a.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def rom_batch(a, P, W):
    """Reduced models beyond the CFL limit, many at once: 2-D 96 x 96 lossless
    PEC cavities (1 mm, eps_r ~ U[1,6] on 8 x 8 blocks, seed 1000 + i, one
    port + one probe), q_i = 5 round(U[50,400]/5) (seed 2), FP32 reductions,
    clamp at s = 4.95, then a.rom_steps FP32 steps of all models in one
    rom_step launch (timed with HIP events on the launch stream)."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    n = a.models
    orders = W.rom_batch_orders(2, n)
    roms, wls = [], []
    t = time.perf_counter()
    for i in range(n):
        wl = W.cavity2d(nx=96, ny=96, d=1e-3, seed=1000 + i, eps_block=8, eps_range=(1, 6),
                        f0=10e9, bw=10e9)
        op = P.Operator.from_workload(wl)
        dt0 = 0.99 * op.dt_max
        roms.append(P.mor_reduce(op, wl.sources, wl.probes, int(orders[i]), dt_ref=dt0,
                                 fmax=20e9, tol=1e-4, defl_tol=1e-6, precision="f32"))
        wls.append(wl)
        if (i + 1) % 16 == 0:
            log(f"[bench] reduced {i + 1}/{n} models ({time.perf_counter() - t:.1f} s)")
    t_reduce = time.perf_counter() - t
    dt = 5 * dt0
    t = time.perf_counter()
    ncl = P.rom_perturb(roms, dt, 0.9999, dtype="f32")
    torch.cuda.synchronize()
    t_perturb = time.perf_counter() - t
    infos = [r.info() for r in roms]
    ns = a.rom_steps
    us = [torch.tensor(W.drive(wl, dt, ns), dtype=torch.float32, device=dev) for wl in wls]
    ys = [torch.zeros((ns, 1), dtype=torch.float32, device=dev) for _ in roms]
    P.rom_step(roms, dt, min(ns, 1000), us, dtype="f32", ys=ys)  # warm-up
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    P.rom_step(roms, dt, ns, us, dtype="f32", ys=ys, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    T = e0.elapsed_time(e1) * 1e-3
    finite = all(bool(torch.isfinite(y).all()) for y in ys)
    q1 = np.array([i["q1"] for i in infos], dtype=np.float64)
    q2 = np.array([i["q2"] for i in infos], dtype=np.float64)
    flop = float(np.sum(4.0 * q1 * q2)) * ns  # A h and A^T e per step
    abytes = float(np.sum(2 * 4.0 * q1 * q2)) * ns  # A (FP32) read twice per step
    # one workgroup (one compute unit) per model: the largest model's matrix
    # stream sets the step time; a CU loads at most 64 B per clock (2.4 GHz)
    big = int(np.argmax(q1 * q2))
    cu_gbs = 2 * 4.0 * q1[big] * q2[big] * ns / T / 1e9
    cu_peak = 64 * 2.4
    out = {
        "metric": "reduced-model steps/s", "value": round(n * ns / T, 1),
        "unit": "model-steps/s", "n_gpus": 1, "steps": ns, "warmup": 1,
        "ms_per_step": round(T / ns * 1e3, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{n} reduced models of 96x96 lossless 2-D cavities, "
                               f"q=5*round(U[50,400]/5), clamp and {ns} steps at s=4.95 in one launch",
                   "models": n, "q_sum": int(q1.sum()), "parallelism": "single GPU"},
        # the stepping matrices of all models (~125 MB in FP32) stay in the
        # 256 MB Infinity Cache, so the aggregate rate is quoted against HBM for
        # scale only; what bounds the step is the load rate of the compute unit
        # that streams the largest model
        "roofline": {"bound": "hbm", "achieved": round(abytes / T / 1e9, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(abytes / T / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None, "cache_resident": True,
                     "largest_model": {"q1": int(q1[big]), "q2": int(q2[big]),
                                       "cu_load_gbs": round(cu_gbs, 1), "cu_peak_gbs": cu_peak,
                                       "frac": round(cu_gbs / cu_peak, 3)},
                     "fp_tflops": round(flop / T / 1e12, 3)},
        "breakdown": {"t_reduce_s": round(t_reduce, 2), "t_perturb_s": round(t_perturb, 3),
                      "t_step_s": round(T, 4), "n_clamped": int(sum(ncl)),
                      "certified": all(i["guard_margin"] > 0 for i in infos),
                      "finite": finite},
    }
    print(json.dumps(out), flush=True)


def cavity256(a, P, W):
    """256^3 lossy cavity (the 128^3 recipe at twice the size: eps_r ~ U[1,4],
    sigma_e ~ U[0, 0.01] S/m on 8^3 blocks, seed 1), 16 z-directed ports: 500
    FP32 leapfrog steps, then a block Krylov sweep with the 16 ports as one
    block of right-hand sides: four block steps at the complex point
    z1 = M exp(j 2 pi f_max dt) (the conjugate pair alone, q = 128: 64 complex
    columns, 128 real after the split), FP32 COCG to 1e-4, FP64 CGS2 of each
    block against the accumulated basis, deflating CholQR2 of V1 and V2 and
    the projection.  The field state (400 MB) and the Krylov vectors (6.5 GB
    per 16-column block vector) stream from HBM; the point basis takes 104 GB
    and V1 + V2 another 104 GB, allocated once the solver's vectors are freed."""
    import torch
    dev = torch.device("cuda:0")
    n = 256
    wl = W.cavity3d(n=n, d=1e-3, seed=1, block=8, nports=16, f0=1.5e9, bw=1.5e9)
    ncells = n ** 3
    op = P.Operator.from_workload(wl)
    dt = 0.99 * op.dt_max
    nfull = 500
    signs = W.port_signs(1, 16)
    u = torch.tensor(W.drive(wl, dt, nfull, signs), dtype=torch.float32, device=dev)
    f32 = op.new_fields(torch.float32)
    y = torch.zeros((nfull, 16), dtype=torch.float32, device=dev)
    P.fdtd_step(op, dt, 20, f32, wl.sources, u[:20], wl.probes, y[:20])  # warm-up
    torch.cuda.synchronize()
    P.yeerom.profile_reset()
    P.yeerom.profile_enable(True)
    t = time.perf_counter()
    P.fdtd_step(op, dt, nfull, f32, wl.sources, u, wl.probes, y)
    torch.cuda.synchronize()
    t_fdtd = time.perf_counter() - t
    log("[bench] cavity256: 16-RHS block sweep, four block steps at z1")
    t = time.perf_counter()
    rom = P.mor_reduce(op, wl.sources, wl.probes, 128, dt_ref=dt, fmax=3e9, M=1.1, tol=1e-4,
                       max_iter=4000, defl_tol=1e-6, precision="f32", pair_only=True)
    torch.cuda.synchronize()
    t_red = time.perf_counter() - t
    P.yeerom.profile_enable(False)
    info = rom.info()
    kernels = {}
    for name in ("fdtd_e", "fdtd_h", "fdtd_fused", "cocg_fused", "cocg_fused_real"):
        cnt, ms = P.yeerom.profile_read(name)
        kernels[name] = {"launches": cnt, "ms_total": round(ms, 2), "us_avg": round(1e3 * ms / max(cnt, 1), 2)}
    nb = info["matvecs"] / max(info["solve_iters"], 1)  # active columns per pass (of 16)
    per_launch = {"fdtd_e": 36.0 * ncells, "fdtd_h": 36.0 * ncells, "fdtd_fused": 48.0 * ncells,
                  "cocg_fused": (180.0 * nb + 27.0) * ncells,
                  "cocg_fused_real": (90.0 * nb + 15.0) * ncells}
    roof = {}
    copy_gbs = copy_ceiling_gbs()
    for k_, b_ in per_launch.items():
        us = kernels[k_]["us_avg"]
        if kernels[k_]["launches"]:
            gbs = b_ / (us * 1e-6) / 1e9
            roof[k_] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_launch": b_, "us_per_launch": us,
                        "copy_ceiling_gbs": copy_gbs, "frac_of_copy": round(gbs / copy_gbs, 4),
                        # counters taken on this workload's leapfrog only
                        "traffic": (measured_traffic("fdtd_fused_256") if k_ == "fdtd_fused" else
                                    measured_traffic("cocg_fused_256", b_) if k_ == "cocg_fused"
                                    else None)}
    cell_updates = ncells * nfull + ncells * info["matvecs"]
    out = {
        "metric": "Gcell-updates/s (FDTD+Krylov), 256^3", "value": round(cell_updates / (t_fdtd + t_red) / 1e9, 3),
        "unit": "Gcell-updates/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round((t_fdtd + t_red) * 1e3, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "3-D lossy PEC cavity 256^3 cells 1 mm, 16 ports; 500 FP32 leapfrog "
                               "steps + 16-RHS block Krylov sweep (4 block steps at z1, q=128)",
                   "cells": ncells, "parallelism": "single GPU"},
        "kernels": kernels, "roofline": roof,
        "breakdown": {"t_fdtd_s": round(t_fdtd, 3), "fdtd_gcells": round(ncells * nfull / t_fdtd / 1e9, 2),
                      "t_reduce_s": round(t_red, 3), "solve_s": round(info["seconds_solve"], 3),
                      "orth_s": round(info["seconds_orth"], 3), "project_s": round(info["seconds_project"], 3),
                      "cocg_iters": info["solve_iters"], "matvecs": info["matvecs"],
                      "q1": info["q1"], "q2": info["q2"], "relres_max": info["relres_max"],
                      "torch_mem_peak_gb": round(torch.cuda.max_memory_allocated() / 1e9, 2)},
    }
    print(json.dumps(out), flush=True)


def adjoint_design(a, P, W):
    """Differentiation workload: 2-D 512 x 512 PEC box, 0.5 mm cells, a 128 x 128
    design region with per-cell eps_r ~ U[1,4] and sigma_e ~ U[0, 0.01] S/m and
    PEC strips 2 cells wide every 16; 3000 steps; J = dt sum_n y_n^2 at one
    probe.  fdtd_adjoint runs the forward leapfrog (checkpoint every 64 steps),
    then the reverse sweep recomputing each segment, and accumulates dJ/d eps_r
    and dJ/d sigma_e per cell.  FP32 timed (3 warm runs, median); FP64 once for
    the accuracy of the FP32 gradient."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    wl = W.design2d()
    op = P.Operator.from_workload(wl)
    dt = 0.99 * op.dt_max
    nsteps, ck = 3000, 64
    ncells = wl.nx * wl.ny
    grads, times = {}, {}
    for prec, tdt in (("f32", torch.float32), ("f64", torch.float64)):
        u = torch.tensor(W.drive(wl, dt, nsteps), dtype=tdt, device=dev)
        f = op.new_fields(tdt)
        y = torch.zeros((nsteps, 1), dtype=tdt, device=dev)
        P.fdtd_step(op, dt, nsteps, f, wl.sources, u, wl.probes, y)
        dJdy = (2.0 * dt * y).contiguous()
        runs = []
        for _ in range(3 if prec == "f32" else 1):
            torch.cuda.synchronize()
            t = time.perf_counter()
            ge, gs = P.yeerom.fdtd_adjoint(op, dt, nsteps, wl.sources, u, wl.probes, dJdy, ck)
            torch.cuda.synchronize()
            runs.append(time.perf_counter() - t)
        times[prec] = sorted(runs)[len(runs) // 2]
        grads[prec] = (ge.cpu().numpy(), gs.cpu().numpy())
    c0 = (wl.nx - 128) // 2
    reg = (slice(c0, c0 + 128), slice(c0, c0 + 128))
    rel = lambda a_, b_: float(np.linalg.norm(a_[reg] - b_[reg]) / np.linalg.norm(b_[reg]))
    T = times["f32"]
    # forward (checkpointed) + recomputation + adjoint: 3 leapfrog sweeps of nsteps
    out = {
        "metric": "adjoint gradient: cell-steps/s (forward + recompute + reverse)",
        "value": round(3 * ncells * nsteps / T / 1e9, 3), "unit": "Gcell-steps/s", "n_gpus": 1,
        "steps": nsteps, "warmup": 0, "ms_per_step": round(T / nsteps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2-D 512x512 PEC box, 128x128 design region (per-cell eps_r, sigma_e), "
                               "PEC strips, 3000 steps, checkpoint every 64",
                   "cells": ncells, "parallelism": "single GPU"},
        "breakdown": {"t_grad_f32_s": round(T, 4), "t_grad_f64_s": round(times["f64"], 4),
                      "grad_eps_f32_vs_f64": rel(grads["f32"][0], grads["f64"][0]),
                      "grad_sigma_f32_vs_f64": rel(grads["f32"][1], grads["f64"][1]),
                      "n_parameters": 2 * 128 * 128},
    }
    print(json.dumps(out), flush=True)


def board(a, P, W):
    """Graded-mesh board, 256 x 128 x 64 cells: 1 mm in x and y, 0.1 mm in z for
    the 8 substrate cells (eps_r 3.38), 1 mm above; PEC strip on node plane 8,
    y in [62, 66), x in [16, 240); two 8-edge line ports; pulse f0 = 3 GHz,
    BW 3 GHz, f_max 6 GHz (about 130 modes of the closed box in band; a 10 GHz /
    10 GHz pulse excites ~4,600, beyond what q = 300 can represent); expansion
    radius M = 1.02 (see below).
    Reference: FP64 full-order leapfrog, 20,000 steps at 0.99 of
    the fine-cell CFL step.  Reduction q = 300 (L = 2, M = 1.1, FP32 solves to
    1e-4), clamp and 2,000 FP32 reduced steps at s = 9.9; probe error on every
    10th reference sample; FP64 reduced adjoint of J = dt sum y^2 with respect
    to the substrate eps_r (basis frozen), against central differences."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    wl = W.board3d(f0=3e9, bw=3e9)
    fmax = wl.f0 + wl.bw
    op = P.Operator.from_workload(wl)
    dt = 0.99 * op.dt_max
    nfull, kfac = 20_000, 10
    u64 = torch.tensor(W.drive(wl, dt, nfull), dtype=torch.float64, device=dev)
    f64 = op.new_fields(torch.float64)
    y_ref = torch.zeros((nfull, 2), dtype=torch.float64, device=dev)
    log("[bench] board: FP64 reference")
    torch.cuda.synchronize()
    t = time.perf_counter()
    P.fdtd_step(op, dt, nfull, f64, wl.sources, u64, wl.probes, y_ref)
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t
    y_ref = y_ref.cpu().numpy()
    log("[bench] board: reduction q=300")
    t = time.perf_counter()
    # expansion radius: the fine cells fix dt, so 2 pi f_max dt is only 0.012 and
    # M = 1.1 puts every point far outside the band (s = ln M / dt ~ 8x the band
    # edge; measured ROM error O(1) on a 64x32x20 board).  M = 1.02 (ln M ~ 1.6 x
    # 2 pi f_max dt) brings the points next to the band while the FP32 shifted
    # solves still converge to 1e-4 (M = exp(2 pi f_max dt) stalls above it).
    M = 1.02
    rom = P.mor_reduce(op, wl.sources, wl.probes, 300, dt_ref=dt, fmax=fmax, M=M, L=2, tol=1e-4,
                       max_iter=40000, defl_tol=1e-6, precision="f32")
    torch.cuda.synchronize()
    t_red = time.perf_counter() - t
    info = rom.info()
    rows = []
    for k in (1, 2, 5, 10):
        dtr, nr = k * dt, nfull // k
        u = torch.tensor(W.drive(wl, dtr, nr), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        ncl = P.rom_perturb(rom, dtr, 0.9999, dtype="f32")
        y = P.rom_step([rom], dtr, nr, [u], dtype="f32")[0]
        torch.cuda.synchronize()
        t_run = time.perf_counter() - t
        y = y.cpu().numpy().astype(np.float64)
        ref = y_ref[k - 1::k][:nr]
        rows.append({"s": round(0.99 * k, 2), "n_clamped": int(ncl), "t_s": round(t_run, 4),
                     "err": float(np.linalg.norm(y - ref) / np.linalg.norm(ref))})
    log("[bench] board: reduced adjoint vs central differences")
    dtr, nr = kfac * dt, nfull // kfac
    slab = np.zeros_like(wl.eps_r)
    slab[:8] = 1.0
    dDe = P.yeerom.rom_project_cells(op, rom, slab, "eps")
    m = rom.matrices()
    u = torch.tensor(W.drive(wl, dtr, nr), dtype=torch.float64, device=dev)

    def J_of(theta):
        r = P.Rom.from_matrices(m["De"] + theta * dDe, m["Dm"], m["K"], m["B1"], m["L1"],
                                Dse=m["Dse"], Dsm=m["Dsm"], B2=m["B2"], L2=m["L2"])
        n = P.rom_perturb(r, dtr, 0.9999, dtype="f64")
        y = P.rom_step([r], dtr, nr, [u], dtype="f64")[0]
        return float(dtr * (y ** 2).sum()), n, y

    J0, n0, y0 = J_of(0.0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    through = info["q1"] == info["q2"]  # the clamp derivative needs a square A
    res = P.yeerom.rom_adjoint(rom, dtr, nr, u, (2 * dtr * y0).contiguous(), dDe=dDe,
                               through_clamp=through)
    t_adj = time.perf_counter() - t
    if not through:
        res["dJ"] = res["dJ_frozen"]
    h = 1e-4
    (jp, n1, _), (jm, n2, _) = J_of(h), J_of(-h)
    fd = (jp - jm) / (2 * h)
    # headline: the largest s whose probe error meets 1e-3 (as for the cavity);
    # none may qualify, and then there is no speedup at the metric's accuracy
    ok = [r for r in rows if r["err"] <= 1e-3]
    best = max(ok, key=lambda r: r["s"]) if ok else None
    speedup = round(t_full / (t_red + best["t_s"]), 4) if best else None
    out = {
        "metric": ("end-to-end speedup vs FP64 full-order FDTD at the largest s with probe "
                   "error <= 1e-3" + ("" if best else " (no s meets 1e-3: null)")),
        "value": speedup, "s_at_1e-3": best["s"] if best else None,
        "unit": "x", "n_gpus": 1, "steps": nfull, "warmup": 0, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "graded-mesh board 256x128x64 (0.1 mm substrate under 1 mm air), "
                               "2 line ports, pulse 3+-3 GHz, q=300, clamp and step at s=0.99..9.9",
                   "cells": 256 * 128 * 64, "q": 300, "parallelism": "single GPU"},
        "breakdown": {"t_full_fp64_s": round(t_full, 3), "t_reduce_s": round(t_red, 3), "M": M,
                      "q1": info["q1"], "q2": info["q2"], "cocg_iters": info["solve_iters"],
                      "relres_max": info["relres_max"], "sweep": rows,
                      "adjoint": {"J": J0, "dJ_adjoint": res["dJ"], "dJ_fd": fd,
                                  "rel_mismatch": abs(res["dJ"] - fd) / abs(fd),
                                  "n_clamped": int(n0), "clamp_set_stable": n1 == n2 == n0,
                                  "through_clamp": through,
                                  "t_adjoint_s": round(t_adj, 3)}},
    }
    print(json.dumps(out), flush=True)


def iris(a, P, W):
    """The 2-D waveguide filter of Sec. V-B: 41 x 401 cells of 1.25 mm, eps_r
    2.5, five PEC irises, 5-cell matched absorbers, line source at one end, line
    probe at the other; pulse f0 = 1.5 GHz, bandwidth 3 GHz.  Reference: FP64
    full-order leapfrog, 20,000 steps at s = 0.99 (as in Sec. V-B), and the same
    run of the guide without irises for S21 = Y_filter / Y_empty over the
    propagating band 2-4.5 GHz.  Reduced models: q = 200, five points, FP32
    COCG to 1e-4, at the paper's M = 1.1 (f_max = 3 GHz) and at M = 1.02
    (f_max = f0 + BW = 4.5 GHz, FP64 solves); clamp and FP32 stepping at
    s = 0.99, 4.95, 8.91; waveform and S21 errors against the reference."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    wl = W.iris_guide2d()
    empty = W.iris_guide2d(n_iris=0)
    op = P.Operator.from_workload(wl)
    op0 = P.Operator.from_workload(empty)
    dt = 0.99 * op.dt_max
    nfull = 20_000
    u64 = torch.tensor(W.drive(wl, dt, nfull), dtype=torch.float64, device=dev)
    freqs = np.linspace(2.0e9, 4.5e9, 126)

    def fdtd(o):
        f = o.new_fields(torch.float64)
        y = torch.zeros((nfull, 1), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        P.fdtd_step(o, dt, nfull, f, wl.sources, u64, wl.probes, y)
        torch.cuda.synchronize()
        return y, time.perf_counter() - t

    log("[bench] iris: FP64 references")
    y_ref, t_full = fdtd(op)
    y_emp, _ = fdtd(op0)
    Ye = P.yeerom.probe_dft(y_emp, dt, freqs, t0=dt).cpu().numpy()[:, 0]
    s21_ref = P.yeerom.probe_dft(y_ref, dt, freqs, t0=dt).cpu().numpy()[:, 0] / Ye
    y_ref = y_ref.cpu().numpy()
    runs = []
    # M = 1.02 brings the points 5x closer to the unit circle: the shifted
    # systems are ~25x worse conditioned and FP32 COCG stalls above 1e-4 there,
    # so those solves run in FP64 (46k unknowns: cheap either way)
    for M, fmax, prec in ((1.1, 3e9, "f32"), (1.02, wl.f0 + wl.bw, "f64")):
        log(f"[bench] iris: reduction q=200 M={M} ({prec} solves)")
        torch.cuda.synchronize()
        t = time.perf_counter()
        rom = P.mor_reduce(op, wl.sources, wl.probes, 200, dt_ref=dt, fmax=fmax, M=M, L=2,
                           tol=1e-4, max_iter=40000, defl_tol=1e-6, precision=prec)
        torch.cuda.synchronize()
        t_red = time.perf_counter() - t
        info = rom.info()
        rows = []
        for k in (1, 5, 9):
            dtr, nr = k * dt, nfull // k
            u = torch.tensor(W.drive(wl, dtr, nr), dtype=torch.float32, device=dev)
            torch.cuda.synchronize()
            t = time.perf_counter()
            ncl = P.rom_perturb(rom, dtr, 0.9999, dtype="f32")
            y = P.rom_step([rom], dtr, nr, [u], dtype="f32")[0]
            torch.cuda.synchronize()
            t_run = time.perf_counter() - t
            s21 = P.yeerom.probe_dft(y, dtr, freqs, t0=dtr).cpu().numpy()[:, 0] / Ye
            y = y.cpu().numpy().astype(np.float64)
            ref = y_ref[k - 1::k][:nr]
            rows.append({"s": round(0.99 * k, 2), "n_clamped": int(ncl), "t_s": round(t_run, 4),
                         "err": float(np.linalg.norm(y - ref) / np.linalg.norm(ref)),
                         "s21_err": float(np.max(np.abs(s21 - s21_ref)))})
        runs.append({"M": M, "fmax_hz": fmax, "solve_dtype": prec, "t_reduce_s": round(t_red, 3),
                     "q1": info["q1"],
                     "q2": info["q2"], "cocg_iters": info["solve_iters"],
                     "relres_max": info["relres_max"], "sweep": rows})
    ok = [(r, run) for run in runs for r in run["sweep"] if r["err"] <= 1e-3]
    best = max(ok, key=lambda x: x[0]["s"]) if ok else None
    speedup = (round(t_full / (best[1]["t_reduce_s"] + best[0]["t_s"]), 4) if best else None)
    out = {
        "metric": ("end-to-end speedup vs FP64 full-order FDTD at the largest s with probe "
                   "error <= 1e-3" + ("" if best else " (no reduced model meets 1e-3: null)")),
        "value": speedup, "unit": "x", "n_gpus": 1, "steps": nfull, "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "2-D waveguide filter 41x401 cells of 1.25 mm, eps_r 2.5, five "
                               "irises, matched absorbers, line source and probe 380 cells "
                               "apart; q=200, clamp and step at s=0.99, 4.95, 8.91",
                   "cells": 41 * 401, "q": 200, "parallelism": "single GPU"},
        "breakdown": {"t_full_fp64_s": round(t_full, 3), "s21_band_hz": [2.0e9, 4.5e9],
                      "s21_ref_abs_range": [float(np.abs(s21_ref).min()),
                                            float(np.abs(s21_ref).max())],
                      "runs": runs},
    }
    print(json.dumps(out), flush=True)


def accuracy(P, W, wl, op, signs, dt, nfull, q, mor_kw):
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    u64 = torch.tensor(W.drive(wl, dt, nfull, signs), dtype=torch.float64, device=dev)
    f64 = op.new_fields(torch.float64)
    y_ref = torch.zeros((nfull, 4), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    P.fdtd_step(op, dt, nfull, f64, wl.sources, u64, wl.probes, y_ref)
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t
    y_ref = y_ref.cpu().numpy()
    torch.cuda.synchronize()
    t = time.perf_counter()
    rom = P.mor_reduce(op, wl.sources, wl.probes, q, **mor_kw)
    torch.cuda.synchronize()
    t_red = time.perf_counter() - t
    rows = []
    for k in (1, 2, 3, 5):
        dtr = k * dt
        nr = nfull // k
        u = torch.tensor(W.drive(wl, dtr, nr, signs), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        ncl = P.rom_perturb(rom, dtr, 0.9999, dtype="f32")
        y = P.rom_step([rom], dtr, nr, [u], dtype="f32")[0]
        torch.cuda.synchronize()
        t_run = time.perf_counter() - t
        y = y.cpu().numpy().astype(np.float64)
        ref = y_ref[k - 1::k][:nr]
        err = float(np.linalg.norm(y - ref) / np.linalg.norm(ref))
        rows.append({"s": round(0.99 * k, 2), "err": err, "n_clamped": int(ncl),
                     "t_perturb_step_s": round(t_run, 4),
                     "t_mor_total_s": round(t_red + t_run, 4)})
    ok = [r for r in rows if r["err"] <= 1e-3]
    best = max(ok, key=lambda r: r["s"]) if ok else None
    # reduction time against Krylov work: the shifted solves stopped at larger
    # normalised residuals than Sec. IV-B's 1e-4, and the probe error that
    # leaves at s = 0.99 and 2.97
    curve = []
    for tol in (1e-4, 3e-4, 1e-3, 3e-3):
        kw = dict(mor_kw, tol=tol)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r_ = P.mor_reduce(op, wl.sources, wl.probes, q, **kw)
        torch.cuda.synchronize()
        tr = time.perf_counter() - t
        inf = r_.info()
        row = {"tol": tol, "cocg_iters": inf["solve_iters"], "matvecs": inf["matvecs"],
               "t_reduce_s": round(tr, 4), "t_solve_s": round(inf["seconds_solve"], 4),
               "t_orth_s": round(inf["seconds_orth"], 4)}
        for k in (1, 3):
            dtr, nr = k * dt, nfull // k
            u = torch.tensor(W.drive(wl, dtr, nr, signs), dtype=torch.float32, device=dev)
            P.rom_perturb(r_, dtr, 0.9999, dtype="f32")
            y = P.rom_step([r_], dtr, nr, [u], dtype="f32")[0].cpu().numpy().astype(np.float64)
            ref = y_ref[k - 1::k][:nr]
            row[f"err_s{0.99 * k:.2f}"] = float(np.linalg.norm(y - ref) / np.linalg.norm(ref))
        curve.append(row)
        del r_
    return {"t_full_fp64_s": round(t_full, 4), "t_reduce_s": round(t_red, 4), "sweep": rows,
            "s_at_1e-3": best["s"] if best else None,
            "speedup": round(t_full / best["t_mor_total_s"], 3) if best else None,
            "break_even_steps": None if not best else
            int(math.ceil(best["t_mor_total_s"] / (t_full / nfull))),
            "tol_curve": curve}


def cpu_baseline():
    """The FP64 oracle on bounded samples of the same recipe: its leapfrog
    (the metric's unit) and its reduction (the step's other leg)."""
    import numpy as np

    import workloads as W
    from oracle import yee
    n, steps = 40, 400
    wl = W.cavity3d(n=n, d=1e-3, seed=1, block=8, nports=4, margin=4)
    op = yee.assemble(wl)
    dt = 0.99 * yee.cfl_dt_max(op.grid)
    B = yee.port_matrix(op, wl.sources, True)
    L = yee.port_matrix(op, wl.probes, False)
    u = W.drive(wl, dt, steps)
    times = []
    for _ in range(3):
        t = time.perf_counter()
        yee.leapfrog(op, dt, B, u, L)
        times.append(time.perf_counter() - t)
    tm = float(np.median(times))
    return {"value": round(n ** 3 * steps / tm / 1e9, 5), "unit": "Gcell-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"oracle FP64 leapfrog eq.(MNAform) (SciPy sparse, single thread) on a "
                      f"{n}^3-cell cavity of the same material recipe, {steps} steps, median of 3; "
                      f"the oracle's shifted solves are direct (sparse LU) and have no matvec count",
            "host_cores_available": len(os.sched_getaffinity(0)),
            "mor_leg": cpu_baseline_mor()}


def cpu_baseline_mor():
    """One shifted solve and one orthogonalisation pass of the oracle's
    reduction on 12^3 and 16^3 cavities of the benchmark's recipe, and their
    extrapolation to the 128^3 reduction (q = 200: three factorisations, 30
    block solves of 4 right-hand sides, 3 x 180 column projections)."""
    import numpy as np
    import scipy.sparse.linalg as spla

    import workloads as W
    from oracle import mor, yee
    rows = []
    for n in (12, 16):
        wl = W.cavity3d(n=n, d=1e-3, seed=1, block=8, nports=4, margin=3)
        op = yee.assemble(wl)
        dt = 0.99 * yee.cfl_dt_max(op.grid)
        B = yee.port_matrix(op, wl.sources, True).astype(complex)
        z = mor.expansion_points(1.1, 2, wl.f0 + wl.bw, dt)[1]
        P_, Q_ = mor.system_pq(op, dt)
        A = (z * P_ - Q_).tocsc()
        t = time.perf_counter()
        lu = spla.splu(A)
        t1 = time.perf_counter()
        X = lu.solve(B)
        t2 = time.perf_counter()
        rows.append({"n": n, "N": op.N, "lu_s": t1 - t, "solve_s": t2 - t1})
    # one CGS2 pass of a block of 4 complex columns against 36 orthonormal
    # ones (the widest block of a point), on the 16^3 vectors
    N = rows[-1]["N"]
    rng = np.random.default_rng(0)
    Vb = np.linalg.qr(rng.standard_normal((N, 36)) + 1j * rng.standard_normal((N, 36)))[0]
    Wb = rng.standard_normal((N, 4)) + 1j * rng.standard_normal((N, 4))
    t = time.perf_counter()
    for _ in range(2):
        Wb = Wb - Vb @ (Vb.conj().T @ Wb)
    Wb = np.linalg.qr(Wb)[0]
    t_orth = time.perf_counter() - t
    N128 = 6 * 128 ** 3 - 2 * 3 * 128 ** 2  # ~ unknowns of the 128^3 box
    a_lu = math.log(rows[1]["lu_s"] / rows[0]["lu_s"]) / math.log(rows[1]["N"] / rows[0]["N"])
    a_sv = math.log(rows[1]["solve_s"] / rows[0]["solve_s"]) / math.log(rows[1]["N"] / rows[0]["N"])
    r = N128 / rows[1]["N"]
    est = (3 * rows[1]["lu_s"] * r ** a_lu + 30 * rows[1]["solve_s"] * r ** a_sv
           + 3 * 5 * t_orth * r)
    try:
        import threadpoolctl
        blas = max((i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()), default=1)
    except Exception:
        blas = None
    return {"samples": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in x.items()}
                        for x in rows],
            "orth_pass_s": round(t_orth, 4), "lu_exponent": round(a_lu, 2),
            "solve_exponent": round(a_sv, 2),
            "reduction_128_s_extrapolated": round(est, 1), "extrapolated": True,
            "cores": {"lu_and_solve": 1, "orth": blas},
            "note": "SuperLU factorisation of z P - Q (complex, the oracle's direct shifted "
                    "solve) and one block solve at 12^3 and 16^3, power laws in the unknown "
                    "count fitted through the two and extrapolated to the 12.4M unknowns of "
                    "the 128^3 step: an order-of-magnitude estimate (the flop count of a 3-D "
                    "sparse factorisation grows about as N^2 under nested dissection); the "
                    "GPU path solves iteratively instead"}


if __name__ == "__main__":
    main()
