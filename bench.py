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

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2207_04252_amd import synth  # noqa: E402

METRIC = "zone-updates/s per step, FP64 vs FP32-perturbation; adjoint/forward cost ratio"
PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 vector
PEAK_HBM_GBPS = 8000.0    # MI355X HBM3E


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


KERNEL_SOURCES = ("rb_kernels.hip", "rb_device.h", "rb_pert32.h", "rb_internal.h")


def kernel_hash():
    """Hash of the sources the stage kernels are compiled from."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2207_04252_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


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


def timed_rate(rossbi, torch, cfg, precision, steps, warmup):
    """zone-updates/s of `steps` CFL steps after `warmup`, and the per-launch averages of
    the gas and dust stage kernels (HIP events on the library's stream)."""
    xi = synth.noise(cfg)
    sim = rossbi.Sim(cfg, precision=precision, noise=xi)
    del xi
    sim.step(warmup, check=True)
    sim.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps, check=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms, nl = sim.profile_read()
    sim.close()
    return {"zone_updates_per_s": cfg.n_cells * steps / wall, "ms_per_step": 1e3 * wall / steps,
            "gas_kernel_ms": round(float(ms[0]) / max(int(nl[0]), 1), 4),
            "dust_kernel_ms": round(float(ms[1]) / max(int(nl[1]), 1), 4) if nl[1] else None,
            "other_kernels_ms_per_step": round(float(ms[2]) / steps, 4)}


def precision_forms(rossbi, torch, steps):
    """FP64 against the FP32-perturbation form on the one-dust disc, and both on the
    three-dust disc, same GPU, CFL steps."""
    out = {}
    for cfg in (synth.C3_BIFLUID, synth.C4_LARGE):
        n = steps if cfg.n_cells < 3e7 else max(steps // 4, 5)
        log(f"forms: {cfg.name}, {n} steps each")
        r64 = timed_rate(rossbi, torch, cfg, rossbi.RB_FP64, n, 3)
        r32 = timed_rate(rossbi, torch, cfg, rossbi.RB_FP32_PERT, n, 3)
        out[cfg.name] = {"cells": cfg.n_cells, "fields": cfg.n_fields, "steps": n, "fp64": r64,
                         "fp32p": r32,
                         "fp32p_speedup": r32["zone_updates_per_s"] / r64["zone_updates_per_s"]}
    out["fp32p_accuracy"] = ("one step from oracle states, relative per cell: density and "
                             "pressure <= 1e-5 everywhere (measured ~1e-10); dust density "
                             "<= 1e-5 off the midplane layers and on midplane two-cell sums")
    return out


def extensions(rossbi, torch, steps):
    """Cost of the physics beyond the base step on the one-dust disc (FP64, CFL steps):
    indirect gravity (two disc sums per stage), the Epstein / Stokes drag law (per-cell
    stopping times and stiffness partials), the boundary damping zones and the outflow
    z ghosts, each against the base run."""
    base = synth.C3_BIFLUID
    runs = {"base": base, "indirect_gravity": base.with_(indirect=True),
            "epstein_stokes_drag": synth.epstein_grains(base),
            "damping_zones_r_z": base.with_(bc_r=1, bc_z=2),
            "outflow_z": base.with_(bc_z=1)}
    out = {"workload": base.name, "steps": steps}
    r0 = None
    for name, cfg in runs.items():
        log(f"extensions: {name}, {steps} steps")
        r = timed_rate(rossbi, torch, cfg, rossbi.RB_FP64, steps, 3)
        r0 = r0 or r
        r["cost_vs_base"] = round(r["ms_per_step"] / r0["ms_per_step"], 4)
        out[name] = r
    return out


def adjoint_cost(rossbi, torch, steps, ckpt):
    """Forward (rb_step), recorded forward (rb_record) and reverse sweep (rb_adjoint) of
    the same CFL steps on the adjoint disc; the objective is the vortex-core dust mass."""
    cfg = synth.C5_ADJOINT
    xi = synth.noise(cfg)
    log(f"adjoint: {cfg.name}, {steps} steps, checkpoints every {ckpt}")
    sim = rossbi.Sim(cfg, noise=xi)
    sim.step(2, check=True)
    sim.set_fields(sim.fields())  # same state for all three runs below
    x0 = sim.fields()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, dts = sim.step(steps, check=True)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    sim.set_fields(x0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.record(steps, ckpt, dt_list=dts)
    torch.cuda.synchronize()
    t_rec = time.perf_counter() - t0
    lam = np.zeros((cfg.n_fields, cfg.nz, cfg.nr, cfg.nth))
    rc = rossbi.cell_centres_r(cfg)
    th = (np.arange(cfg.nth) + 0.5) * 2 * np.pi / cfg.nth
    core = ((rc >= synth.CORE_R[0]) & (rc <= synth.CORE_R[1]))[:, None] & \
           (np.abs(th - cfg.vortex_th0) < synth.CORE_DTH)[None, :]
    lam[8] = (rossbi.cell_volumes(cfg)[:, None] * core)[None]
    lam_d = torch.as_tensor(lam, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g0, gst = sim.adjoint(lam_d)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    sim.close()
    fwd = 1e3 * t_fwd / steps
    adj = 1e3 * t_adj / steps
    return {"workload": cfg.name, "cells": cfg.n_cells, "steps": steps, "ckpt_every": ckpt,
            "forward_ms_per_step": round(fwd, 4),
            "record_ms_per_step": round(1e3 * t_rec / steps, 4),
            "adjoint_ms_per_step": round(adj, 4),
            "adjoint_over_forward": round(adj / fwd, 3),
            "reverse_only_over_forward": round((adj - fwd) / fwd, 3),
            "note": "adjoint = recompute of each checkpoint segment (one forward step per step) "
                    "+ two transposed stage operators per step; dJ/dSt = %.6e" % gst[0]}


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
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the FP64 / FP32-perturbation comparison on the dust discs")
    ap.add_argument("--forms-steps", type=int, default=40)
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint cost measurement")
    ap.add_argument("--no-extensions", action="store_true",
                    help="skip the indirect-gravity and drag-law cost measurement")
    ap.add_argument("--extensions-steps", type=int, default=40)
    ap.add_argument("--adjoint-steps", type=int, default=200)
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
    sim.close()
    del sim
    if not args.no_forms:
        out["precision_forms"] = precision_forms(rossbi, torch, args.forms_steps)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_cost(rossbi, torch, args.adjoint_steps, 20)
    if not args.no_extensions:
        out["extensions"] = extensions(rossbi, torch, args.extensions_steps)
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(cfg, xi, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
