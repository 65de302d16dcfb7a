#!/usr/bin/env python3
"""Throughput of the RK2 step of the bi-fluid finite-volume scheme on one MI355X.

One step = one full RK2 midpoint step of every cell (two stage launches of the gas
kernel, the dust kernels when present, the CFL/ledger reduction), CFL time step.
The workload is the 3D Keplerian gas disc 128 (r) x 256 (theta) x 64 (z), FP64, with
the seeded vortex and density noise.  Prints one JSON line:

  value          zone-updates/s = cells x steps / wall time of the timed steps
  roofline       the gas stage kernel against the FP64 vector peak: algorithmic FP64
                 operations per launch (counted by the oracle, tests/golden/opcount.json)
                 / average launch time from HIP events on the library's stream; the
                 HBM view (algorithmic bytes 2S read+write in stage 1, 3S in stage 2)
                 rides along; traffic = measured FETCH+WRITE bytes per launch when the
                 counter file in profiles/ matches the current kernel source, else null
  cpu_baseline   the CPU oracle on the host cores, a bounded number of steps of the
                 same workload

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2207_04252_amd import synth  # noqa: E402

METRIC = "zone-updates/s per step, FP64 vs FP32-perturbation; adjoint/forward cost ratio"
PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 vector
PEAK_HBM_GBPS = 8000.0    # MI355X HBM3E


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash():
    p = os.path.join(ROOT, "paper_2207_04252_amd", "csrc", "rb_kernels.hip")
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(workload):
    """FETCH+WRITE bytes per gas-kernel launch from the committed counter summary, if it
    was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"traffic_gas_stage_{workload}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def ops_per_cell_stage(workload):
    p = os.path.join(ROOT, "tests", "golden", "opcount.json")
    with open(p) as f:
        return json.load(f)[workload]["ops_per_cell_stage"]


def cpu_baseline(cfg, xi, budget_s):
    import oracle
    o = oracle.Oracle(cfg, noise=xi)
    n = 0
    t0 = time.perf_counter()
    while True:
        st, _ = o.step(1)
        n += 1
        if st != 0 or time.perf_counter() - t0 > budget_s or n >= 20:
            break
    dt = time.perf_counter() - t0
    threads = oracle.lib().or_threads()
    return {"value": cfg.n_cells * n / dt, "unit": "zone-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n} CFL steps of the full {cfg.nr}x{cfg.nth}x{cfg.nz} workload, FP64, "
                      f"{threads} OpenMP threads ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--calib", action="store_true",
                    help="first copy 256 MiB device to device 3 times (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only (no multi-GPU path); "
              "run with --gpus 1", file=sys.stderr, flush=True)
        sys.exit(2)

    import torch
    from paper_2207_04252_amd import rossbi

    if args.calib:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copies: 3 x 268435456 bytes")
    cfg = synth.C2_DISC
    xi = synth.noise(cfg)
    log(f"init {cfg.name}")
    sim = rossbi.Sim(cfg, noise=xi)
    st, _ = sim.step(args.warmup, check=True)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} steps done")
    sim.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, dts = sim.step(args.steps, check=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ms, nl = sim.profile_read()
    sim.profile(False)
    log(f"timed {args.steps} steps in {wall:.3f} s")

    cells = cfg.n_cells
    value = cells * args.steps / wall
    gas_ms = ms[0] / max(nl[0], 1)
    ops = ops_per_cell_stage(cfg.name)
    achieved = ops * cells / (gas_ms * 1e-3) / 1e12
    S = 8 * cfg.n_fields
    hbm_bytes = 2.5 * S * cells  # mean of 2S (stage 1) and 3S (stage 2) per launch
    hbm = hbm_bytes / (gas_ms * 1e-3) / 1e9
    traffic = measured_traffic(cfg.name)
    roofline = {
        "bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
        "traffic": traffic,
        "kernel": "k_march<gas> (one RK2 stage)", "avg_launch_ms": round(gas_ms, 4),
        "launches": int(nl[0]), "algorithmic_ops_per_cell": round(ops, 1),
        "hbm": {"achieved_GBps": round(hbm, 1), "peak_GBps": PEAK_HBM_GBPS,
                "frac": round(hbm / PEAK_HBM_GBPS, 4),
                "algorithmic_bytes_per_launch": hbm_bytes},
        "other_kernels_ms_per_step": round(float(ms[2]) / args.steps, 4),
    }
    out = {
        "metric": METRIC, "value": value, "unit": "zone-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg.name, "grid": [cfg.nr, cfg.nth, cfg.nz], "cells": cells,
                   "fields": cfg.n_fields, "precision": "fp64", "dt_policy": "cfl",
                   "cfl": cfg.cfl, "sim_time": float(dts.sum())},
        "roofline": roofline,
    }
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(cfg, xi, args.cpu_seconds)
    sim.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
