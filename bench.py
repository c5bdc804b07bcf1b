#!/usr/bin/env python3
"""Throughput of the quasi-cylindrical order-p PSATD PIC cycle on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c1|c0]

A step is one whole PIC cycle (gather + Boris push, cell sort, tile deposit,
forward z-FFT + Hankel transform, current correction + PSATD, inverse
transforms, moving window with injection) over the synthetic beam-plasma
workload, everything resident in HBM.  W untimed steps are followed by K
timed steps; the default W = 1500 puts the timed steps in the steady state of
the 2000-step run, where the wake behind the drive fills the window (the
moving window brings fresh cold plasma in at the head, and before ~1400 steps
part of the box still holds plasma the beam never crossed).  One JSON line is
printed:

  value       = mobile macro-particles x K / wall time  (particle-pushes/s)
  roofline    = the kernel with the largest GPU time, its algorithmic bytes
                (or flops) per launch over its average HIP-event duration
  cpu_baseline= the FP64 oracle on the host cores, one step on a 1/8
                subsample of the same workload, in the same unit
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
MFMA_FP32_TFLOPS = 157.3       # MI355X dense FP32 matrix
MFMA_BF16_TFLOPS = 2500.0      # dense bf16 / fp16

# algorithmic traffic per unit of work (bytes)
BYTES_PER_PARTICLE = {
    # particle record: x, y, z, u_z FP64 (32) + u_x, u_y, q*w FP32 (12) + species (1) = 45 B
    "gather_push": 91.0,   # read x,y,z,u (40) + species (1); write x,y,z,u (40) + key (4); field share ~6
    "sort": 94.0,          # scatter: read key (4) + record (45); write record (45)
    "deposit": 49.0,       # read x,y,z,u (40) + q*w (4); grid share ~5
}
BYTES_PER_CELL = {
    "fft_fwd": 16.0,       # read + write one complex64 per cell and transform
    "fft_inv": 16.0,
    "psatd": 160.0,        # read 11 complex + write 6 complex (E, B) + 3 (J) per cell and mode
}

WORKLOAD_TEXT = {
    "c1": ("beam-driven plasma wakefield at production size: 2048 x 256 cells, 2 azimuthal "
           "modes, stencil order p = 32, dz = 0.02/kp, dr = 0.05/kp, dt = dz/c, moving window; "
           "8,388,608 plasma electrons (2x2x4 per cell) + as many immobile ions; 1e6-particle "
           "1 nC drive and 2e5-particle 50 pC witness, gamma 2000"),
    "c0": ("256 x 64 cells, 2 modes, p = 16, dz = dr = 0.05/kp, moving window; 262,144 plasma "
           "electrons (2x2x4 per cell) + immobile ions; 1e4-particle 100 pC drive, gamma 1000"),
}


def _phase_units(name, wl, n_part, prec):
    """(algorithmic amount per launch, unit, bound, peak) of one timed phase."""
    M, nr, nz = wl.n_modes, wl.nr, wl.nz
    cells = M * nr * nz
    if name in BYTES_PER_PARTICLE:
        return BYTES_PER_PARTICLE[name] * n_part / 1e9, "GB/s", "hbm", HBM_PEAK_GBS
    if name == "fft_fwd":
        return BYTES_PER_CELL[name] * 5 * cells / 1e9, "GB/s", "hbm", HBM_PEAK_GBS
    if name == "fft_inv":
        return BYTES_PER_CELL[name] * 6 * cells / 1e9, "GB/s", "hbm", HBM_PEAK_GBS
    if name == "psatd":
        return BYTES_PER_CELL[name] * nr * nz * M / 1e9, "GB/s", "hbm", HBM_PEAK_GBS
    if name == "scan":          # count read, offset + cursor written, count cleared, per cell key
        return 16.0 * nz * (nr + 1) / 1e9, "GB/s", "hbm", HBM_PEAK_GBS
    if name == "dep_combine":   # 5 source components written, ion background read (2)
        return 8.0 * 7 * cells / 1e9, "GB/s", "hbm", HBM_PEAK_GBS
    if name == "pack":          # 6 field components read and written once
        return 8.0 * 12 * cells / 1e9, "GB/s", "hbm", HBM_PEAK_GBS
    if name in ("dht_fwd", "dht_inv"):
        batch = (5 if name == "dht_fwd" else 6) * M
        flops = 2.0 * nr * nr * (2 * nz) * batch
        peak = MFMA_FP32_TFLOPS if prec == 0 else MFMA_BF16_TFLOPS
        return flops / 1e12, "TFLOP/s", "mfma", peak
    return None


# sources each measured kernel is built from: its traffic record stays valid
# while these files are unchanged
KERNEL_SOURCES = {"deposit": ("deposit.hip", "common.h", "launch.h"),
                  "sort": ("particles.hip", "common.h", "launch.h")}


def _kernel_sources_hash(kernel="deposit"):
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1611_05712_amd", "csrc")
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def _traffic(kernel, workload):
    """HBM GB per launch measured by rocprofv3 FETCH_SIZE / WRITE_SIZE counters,
    each scaled by what it reads for a device copy of known size
    (profiles/traffic.json); None once the kernel sources have changed."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    e = d.get(workload, {}).get(kernel)
    if not e or kernel not in KERNEL_SOURCES or e.get("sources") != _kernel_sources_hash(kernel):
        return None
    return round(e["bytes_per_launch"] / 1e9, 4)


def _cpu_model():
    """Host CPU model as lscpu reports it ('' when lscpu is unavailable)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except Exception:
        return ""
    for line in out.splitlines():
        if line.startswith("Model name:"):
            return line.split(":", 1)[1].strip()
    return ""


def cpu_baseline(wl_name, stride=4):
    """The oracle (never tuned) timed for one PIC step on every `stride`-th
    macro-particle of the workload, in particle-pushes/s: once with the BLAS
    threads the host gives it (the oracle's Hankel products; its particle
    loops are single-threaded NumPy) and once limited to one thread."""
    from oracle.cycle import OracleSim
    from workloads import preset
    from threadpoolctl import threadpool_info, threadpool_limits

    def blas_threads():
        return max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])

    def one_step():
        wl = preset(wl_name)
        for s in wl.species:
            for a in ("x", "y", "z", "ux", "uy", "uz", "w"):
                setattr(s, a, getattr(s, a)[::stride].copy())
            s.w = (s.w * stride).astype(s.w.dtype)
        n_mobile = wl.n_mobile
        o = OracleSim(wl)
        t0 = time.perf_counter()
        o.step(1)
        return n_mobile, time.perf_counter() - t0

    threads = blas_threads()
    n_mobile, dt = one_step()
    with threadpool_limits(limits=1, user_api="blas"):
        _, dt1 = one_step()
    return {"value": n_mobile / dt, "unit": "particle-pushes/s", "cores": int(threads),
            "kind": "oracle",
            "single_core_value": n_mobile / dt1,
            "host_cpus": os.cpu_count(), "cpu_model": _cpu_model(),
            "sample": (f"one full PIC step of the {wl_name} grid with every {stride}th macro-particle "
                       f"({n_mobile} mobile, weights x{stride}): {dt:.1f} s with {threads} BLAS threads "
                       f"(the Hankel products; particle loops are single-threaded NumPy), {dt1:.1f} s on "
                       f"one thread; host has {os.cpu_count()} logical CPUs")}


def scan_bench(args):
    """Scan runs/hour at matched slice energy spread: every run is done twice,
    batched (graph replays, autotuned, BF16x3 split-precision Hankel products)
    and plain (eager steps, FP32 Hankel products, one run at a time); a run
    counts when its final witness slice energy spread agrees within 1 %."""
    import torch
    from paper_1611_05712_amd import Simulation, H_BF16X3, H_FP32
    from paper_1611_05712_amd.scan import run_batched, run_plain, slice_energy_spread
    from workloads import scan_instances, scan_workload
    insts = scan_instances()
    if args.scan > 0:
        insts = insts[:args.scan]
    t0 = time.perf_counter()
    fast, plain = [], []
    for inst in insts:
        wl = scan_workload(inst, args.scan_steps)
        fast.append(Simulation.from_workload(wl, hankel_prec=H_BF16X3, device="cuda:0"))
        plain.append(Simulation.from_workload(wl, hankel_prec=H_FP32, device="cuda:0"))
        del wl
        print(f"init {inst.index}: nz {inst.nz} nr {inst.nr} p {inst.order}", file=sys.stderr, flush=True)
    init_s = time.perf_counter() - t0
    plain_s = 0.0
    for k, s in enumerate(plain):
        plain_s += run_plain(s, args.scan_steps)
        print(f"plain {k}: {plain_s:.2f} s", file=sys.stderr, flush=True)
    b = run_batched(fast, args.scan_steps)
    rows, matched = [], 0
    for inst, f, p in zip(insts, fast, plain):
        ef, ep = slice_energy_spread(f), slice_energy_spread(p)
        ok = bool(abs(ef - ep) <= 0.01 * abs(ep))   # False when either is NaN
        dw = p.diagnostics("witness", slice_len=0.02975, allow_nan=True)
        matched += int(ok)
        rows.append({"run": inst.index, "order": inst.order, "nz": inst.nz, "nr": inst.nr,
                     "dz": round(inst.dz, 5), "dr": round(inst.dr, 5), "gamma_w": round(inst.gamma_w, 1),
                     "spread_batched": ef, "spread_plain": ep, "matched": ok,
                     "witness_live": dw["n"], "witness_slices": dw["n_slices"], "nan_flag": dw["nan_flag"]})
    for s in fast + plain:
        s.close()
    torch.cuda.synchronize()
    n = len(insts)
    out = {"metric": "scan runs/hour at matched slice energy spread (1 %)",
           "value": matched / b["total_s"] * 3600.0, "unit": "runs/hour", "runs": n, "matched": matched,
           "steps": args.scan_steps, "batched_s": round(b["total_s"], 3),
           "batched_note": (f"all {args.scan_steps} steps of every run: per-run autotuning trials, then "
                            f"{b['batch_steps']} steps in one batch ({b['batch_s']:.3f} s); BF16x3 "
                            "Hankel products; device-resident, initialisation excluded"),
           "plain_s": round(plain_s, 3), "plain_runs_per_hour": n / plain_s * 3600.0,
           "init_s": round(init_s, 1), "tunings": b["tunings"], "runs_detail": rows,
           "data": "synthetic", "n_gpus": 1}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=1500)
    ap.add_argument("--workload", default="c1", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--hankel-prec", default="fp32", choices=["fp32", "bf16x3", "fp16x3"])
    ap.add_argument("--damp-cells", type=int, default=0, metavar="N",
                    help="variant: absorbing layers of N cells at both z ends (not the headline line)")
    ap.add_argument("--shape-order", type=int, default=1, choices=[1, 3],
                    help="variant: particle shape (3: cubic B-spline), not the headline line")
    ap.add_argument("--galilean", action="store_true",
                    help="variant: Galilean field update in coordinates moving with the window (not the headline line)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eager", action="store_true",
                    help="time eager steps instead of replays of the captured two-step HIP graph")
    ap.add_argument("--scan", type=int, default=0, metavar="N",
                    help="instead of the c1 bench: the parameter scan (first N runs of the "
                         "64-run scan, 0 = off; -1 = all), batched with split-precision Hankel "
                         "products against plain FP32 runs; prints its own JSON line")
    ap.add_argument("--scan-steps", type=int, default=500)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run 5 device-to-device copies of BYTES (scale of the rocprofv3 "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        n = args.copy_calibration // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        ev[0].record()
        for k in range(5):
            b.copy_(a)
            ev[k + 1].record()
        torch.cuda.synchronize()
        # copies 2-5 (the first one warms up): read + write bytes per time
        ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(1, 5)]
        print(json.dumps({"copy_bytes": 4 * n, "launches": 5, "ms_per_copy": round(sum(ms) / 4, 4),
                          "read_plus_write_TB_s": round(2 * 4 * n / (sum(ms) / 4) / 1e9, 3)}))
        return
    if args.scan:
        scan_bench(args)
        return
    from paper_1611_05712_amd import Simulation
    from workloads import preset

    prec = {"fp32": 0, "bf16x3": 1, "fp16x3": 2}[args.hankel_prec]
    wl = preset(args.workload)
    wl.damp_cells = args.damp_cells
    wl.galilean = args.galilean
    wl.shape_order = args.shape_order
    sim = Simulation.from_workload(wl, hankel_prec=prec, device="cuda:0")
    t0 = time.perf_counter()
    (sim.step if args.eager else sim.step_graph)(args.warmup)
    sim.sync()
    warm_s = time.perf_counter() - t0
    n_before = sim.num_particles()

    # timed region: K whole cycles, no instrumentation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.eager:
        sim.step(args.steps)
    else:
        sim.step_graph(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_after = sim.num_particles()
    n_part = 0.5 * (n_before + n_after)
    # per-kernel durations: the next K cycles with HIP events around every phase
    sim.timing_enable(True)
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    wall_ev = time.perf_counter() - t0
    times = sim.timing_read()
    sim.timing_enable(False)

    cells = wl.nz * wl.nr * wl.n_modes
    spectral_ms = sum(times[k][0] for k in ("fft_fwd", "dht_fwd", "psatd", "dht_inv", "fft_inv",
                                             "pack", "window"))
    kernels = {}
    for name, (tot_ms, nl) in times.items():
        if nl == 0:
            continue
        avg_s = tot_ms / nl / 1e3
        u = _phase_units(name, wl, n_part, prec)
        entry = {"ms_per_launch": round(tot_ms / nl, 5), "launches": nl,
                 "share": round(tot_ms / max(1e-9, sum(t for t, _ in times.values())), 4)}
        if u:
            amount, unit, bound, peak = u
            ach = amount / avg_s
            entry.update({"achieved": round(ach, 2), "unit": unit, "bound": bound,
                          "frac": round(ach / peak, 4)})
        kernels[name] = entry
    dominant = max((k for k in kernels if "achieved" in kernels[k]),
                   key=lambda k: times[k][0])
    d = kernels[dominant]
    peak = _phase_units(dominant, wl, n_part, prec)[3]
    roofline = {"kernel": dominant, "bound": d["bound"], "achieved": d["achieved"], "peak": peak,
                "unit": d["unit"], "frac": d["frac"],
                "traffic": _traffic(dominant, args.workload)}

    out = {
        "metric": "particle-pushes/s (whole PIC cycle) & field cell-updates/s on 1 GPU",
        "value": n_part * args.steps / wall,
        "unit": "particle-pushes/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_TEXT[args.workload]}",
                   "mobile_particles": int(n_part), "cells_per_mode": wl.nz * wl.nr,
                   "modes": wl.n_modes, "order": wl.order,
                   "hankel_prec": args.hankel_prec, "positions": "f64", "damp_cells": args.damp_cells,
                   "galilean": args.galilean, "shape_order": args.shape_order,
                   "stepping": "eager" if args.eager else "hip graph, two steps per replay"},
        "field_cell_updates_per_s": cells * args.steps / (spectral_ms / 1e3) if spectral_ms else None,
        "roofline": roofline,
        "kernels": kernels,
        "kernels_note": (f"HIP-event durations over {args.steps} further cycles "
                         f"({1e3 * wall_ev / args.steps:.3f} ms/step with events)"),
        "warmup_s": round(warm_s, 3),
    }
    sim.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
