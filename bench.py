#!/usr/bin/env python3
"""Throughput of the RK2 step of the bi-fluid finite-volume scheme on one MI355X.

One step = one full RK2 midpoint step of every cell: two stage launches of the gas
kernel and of each dust species' kernel, the CFL/ledger reductions, CFL time step.  The
headline workload is the largest one, 512 (r) x 1024 (theta) x 128 (z), gas plus three
dust species (Stokes numbers 0.01, 0.1, 1), vortex 1e-2 plus density noise 1e-6, in the
FP32-perturbation form (gas deviation and dust velocity deviations stored in FP32 about
the FP64 stationary flow, dust densities in FP64).  Prints one JSON line:

  value          zone-updates/s = cells x steps / wall time of the timed steps
  roofline       the kernel with the largest share of the step (HIP events on the
                 library's stream) against the HBM peak: algorithmic bytes per launch
                 (each stage reads its own fields, the other group's fields for the drag,
                 the base of the update in the second stage, and writes its own fields)
                 / average launch time; traffic = measured FETCH+WRITE bytes per launch
                 when the counter summary in profiles/ was taken on the current kernel
                 source, else null; step_hbm = 5 S bytes per zone-update (S the stored
                 bytes per cell) over the step time
  cpu_baseline   the CPU oracle on the host cores (all threads and one thread) on a
                 radial band of the same workload

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
PEAK_HBM_GBPS = 8000.0    # MI355X HBM3E


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


KERNEL_SOURCES = ("rb_kernels.hip", "rb_device.h", "rb_pert32.h", "rb_internal.h")


def kernel_hash():
    """Hash of the sources the stage kernels are compiled from and of the compiler flags."""
    from paper_2207_04252_amd import build as hipbuild
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2207_04252_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    h.update(" ".join(hipbuild.HIPCC_FLAGS).encode())
    return h.hexdigest()[:16]


def counter_summary(name):
    """A committed counter summary (profiles/<name>.json) if it was taken on the current
    kernel source, else None."""
    p = os.path.join(ROOT, "profiles", f"{name}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return d


def stored_bytes(cfg, fp32p):
    """(gas, each dust species) bytes per cell as stored."""
    if fp32p:
        return 5 * 4, 3 * 4 + 8
    return 5 * 8, 4 * 8


def launch_bytes(cfg, fp32p, group):
    """Algorithmic bytes per cell of one stage launch of a group (mean of the two stages):
    stage 1 reads its fields and writes them, stage 2 also reads the base of the update;
    the drag makes the gas read every dust species and each dust species read the gas."""
    sg, sd = stored_bytes(cfg, fp32p)
    if group == "gas":
        return 2.5 * sg + cfg.n_dust * sd
    return 2.5 * sd + sg


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
    _, dts = sim.step(steps, check=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms, nl = sim.profile_read()
    sim.close()
    return {"zone_updates_per_s": cfg.n_cells * steps / wall, "ms_per_step": 1e3 * wall / steps,
            "wall_s": wall, "sim_time": float(np.sum(dts)),
            "gas_kernel_ms": float(ms[0]) / max(int(nl[0]), 1), "gas_launches": int(nl[0]),
            "dust_kernel_ms": float(ms[1]) / max(int(nl[1]), 1) if nl[1] else None,
            "dust_launches": int(nl[1]),
            "other_kernels_ms_per_step": float(ms[2]) / steps}


def kernel_roofline(cfg, fp32p, r):
    """HBM roofline of the stage kernel with the largest share of the step."""
    tot_gas = r["gas_kernel_ms"] * r["gas_launches"]
    tot_dust = (r["dust_kernel_ms"] or 0.0) * r["dust_launches"]
    group = "gas" if tot_gas >= tot_dust else "dust"
    ms = r["gas_kernel_ms"] if group == "gas" else r["dust_kernel_ms"]
    per_cell = launch_bytes(cfg, fp32p, group)
    bytes_launch = per_cell * cfg.n_cells
    achieved = bytes_launch / (ms * 1e-3) / 1e9
    form = "fp32p" if fp32p else "fp64"
    kname = f"k_march<{group}, {form}>"
    cs = counter_summary(f"counters_{group}_stage_{form}_{cfg.name}")
    traffic = cs["bytes_per_launch"] if cs else None
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
           "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": traffic,
           "kernel": kname + " (one RK2 stage)", "avg_launch_ms": round(ms, 4),
           "share_of_step": round(max(tot_gas, tot_dust) / (r["ms_per_step"] * r["steps"]), 3),
           "algorithmic_bytes_per_cell_launch": per_cell,
           "algorithmic_bytes_per_launch": bytes_launch}
    if cs and "valu" in cs:
        out["valu"] = cs["valu"]
    return out


def step_hbm(cfg, fp32p, ms_per_step):
    sg, sd = stored_bytes(cfg, fp32p)
    S = sg + cfg.n_dust * sd
    gbps = 5 * S * cfg.n_cells / (ms_per_step * 1e-3) / 1e9
    return {"bytes_per_zone_update": 5 * S, "achieved_GBps": round(gbps, 1),
            "frac": round(gbps / PEAK_HBM_GBPS, 4)}


def precision_forms(rossbi, torch, steps):
    """FP64 against the FP32-perturbation form on the one-dust and three-dust discs, same
    GPU, CFL steps."""
    out = {}
    for cfg in (synth.C3_BIFLUID, synth.C4_LARGE):
        n = steps if cfg.n_cells < 3e7 else max(steps // 2, 5)
        log(f"forms: {cfg.name}, {n} steps each")
        res = {}
        for prec, nm in ((rossbi.RB_FP64, "fp64"), (rossbi.RB_FP32_PERT, "fp32p")):
            r = timed_rate(rossbi, torch, cfg, prec, n, 3)
            r["steps"] = n
            res[nm] = {"zone_updates_per_s": r["zone_updates_per_s"],
                       "ms_per_step": round(r["ms_per_step"], 4),
                       "gas_kernel_ms": round(r["gas_kernel_ms"], 4),
                       "dust_kernel_ms": round(r["dust_kernel_ms"], 4),
                       "step_hbm": step_hbm(cfg, nm == "fp32p", r["ms_per_step"])}
        res["fp32p_speedup"] = res["fp32p"]["zone_updates_per_s"] / res["fp64"]["zone_updates_per_s"]
        res["cells"] = cfg.n_cells
        out[cfg.name] = res
    out["fp32p_accuracy"] = (
        "bi-fluid slice 36x80x64, 500 steps against the FP64 oracle: density and pressure "
        "<= 1e-5 relative per cell (tests/test_gpu_fp32p.py)")
    return out


def extensions(rossbi, torch, steps):
    """Cost of the physics beyond the base step on the one-dust disc (FP64, CFL steps):
    indirect gravity, the Epstein / Stokes drag law, the boundary damping zones and the
    outflow z ghosts, each against the base run."""
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
        out[name] = {"ms_per_step": round(r["ms_per_step"], 4),
                     "cost_vs_base": round(r["ms_per_step"] / r0["ms_per_step"], 4)}
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
    geo = sim.geometry()
    th = (np.arange(cfg.nth) + 0.5) * 2 * np.pi / cfg.nth
    core = ((geo["rc"] >= synth.CORE_R[0]) & (geo["rc"] <= synth.CORE_R[1]))[:, None] & \
           (np.abs(th - cfg.vortex_th0) < synth.CORE_DTH)[None, :]
    lam = np.zeros((cfg.n_fields, cfg.nz, cfg.nr, cfg.nth))
    lam[8] = (geo["V"][:, None] * core)[None]
    lam = torch.as_tensor(lam, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.adjoint(lam)
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
            "note": "adjoint = recompute of each checkpoint segment (one forward step per step) "
                    "+ two transposed stage operators per step"}


def cpu_baseline(cfg, budget_s):
    """The oracle on a radial band of the workload (full theta and z, the band's own
    log-spaced faces and the workload's seeded noise), all threads, then one thread."""
    import oracle
    nb = 8
    i0 = cfg.nr // 2 - nb // 2
    q = cfg.r_out / cfg.r_in
    band = cfg.with_(nr=nb, r_in=cfg.r_in * q ** (i0 / cfg.nr),
                     r_out=cfg.r_in * q ** ((i0 + nb) / cfg.nr), name=cfg.name + "@band")
    xi = synth.noise(cfg)[:, :, i0:i0 + nb, :].copy()
    nproc = os.cpu_count()
    share = int(os.environ.get("OMP_NUM_THREADS", nproc))  # the host cores this job may use
    out = {}
    for label, threads in (("all", share), ("one", 1)):
        used = oracle.set_threads(threads)
        o = oracle.Oracle(band, noise=xi)
        n = 0
        t0 = time.perf_counter()
        while True:
            st, _ = o.step(1)
            n += 1
            if st != 0 or time.perf_counter() - t0 > budget_s or n >= 50:
                break
        dt = time.perf_counter() - t0
        o.close()
        out[label] = {"value": band.n_cells * n / dt, "threads": used, "steps": n, "seconds": dt}
    oracle.set_threads(share)
    a, b = out["all"], out["one"]
    return {"value": a["value"], "unit": "zone-updates/s", "cores": a["threads"],
            "kind": "oracle", "nproc": nproc,
            "one_thread_value": b["value"],
            "sample": f"radial band of {nb} rows x {cfg.nth} x {cfg.nz} ({band.n_cells} cells, "
                      f"r in [{band.r_in:.4f}, {band.r_out:.4f}]) of the {cfg.nr}x{cfg.nth}x"
                      f"{cfg.nz} workload, FP64, CFL steps: {a['steps']} steps on "
                      f"{a['threads']} OpenMP threads ({a['seconds']:.1f} s), {b['steps']} on "
                      f"1 thread ({b['seconds']:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the FP64 / FP32-perturbation comparison on the dust discs")
    ap.add_argument("--forms-steps", type=int, default=20)
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint cost measurement")
    ap.add_argument("--no-extensions", action="store_true",
                    help="skip the cost of the optional physics")
    ap.add_argument("--extensions-steps", type=int, default=20)
    ap.add_argument("--adjoint-steps", type=int, default=200)
    ap.add_argument("--headline-only", action="store_true",
                    help="time the headline workload only (for profiling)")
    ap.add_argument("--calib", action="store_true",
                    help="first write and read 1 GiB (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only (no multi-GPU path); "
              "run with --gpus 1", file=sys.stderr, flush=True)
        sys.exit(2)

    import torch
    from paper_2207_04252_amd import rossbi

    if args.calib:
        # counter calibration: a fill kernel writing 1 GiB, then two reduction kernels
        # reading it (the buffer is four times the 256 MB last-level cache)
        src = torch.ones(256 << 20, dtype=torch.float32, device="cuda")
        tot = [float(src.sum()) for _ in range(2)]
        torch.cuda.synchronize()
        del src
        log(f"calibration: fill 1073741824 bytes, read it twice (sum {tot[0]:.0f})")
    cfg = synth.C4_LARGE
    log(f"headline {cfg.name}, FP32-perturbation form, {args.warmup} + {args.steps} steps")
    r = timed_rate(rossbi, torch, cfg, rossbi.RB_FP32_PERT, args.steps, args.warmup)
    r["steps"] = args.steps
    log(f"timed {args.steps} steps in {r['wall_s']:.3f} s")
    value = r["zone_updates_per_s"]
    out = {
        "metric": METRIC, "value": value, "unit": "zone-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": cfg.name, "grid": [cfg.nr, cfg.nth, cfg.nz], "cells": cfg.n_cells,
                   "fields": cfg.n_fields, "precision": "fp32-perturbation", "dt_policy": "cfl",
                   "cfl": cfg.cfl, "sim_time": r["sim_time"]},
        "roofline": kernel_roofline(cfg, True, r),
        "step_hbm": step_hbm(cfg, True, r["ms_per_step"]),
        "kernels": {"gas_ms_per_launch": round(r["gas_kernel_ms"], 4),
                    "dust_ms_per_launch": round(r["dust_kernel_ms"], 4),
                    "other_ms_per_step": round(r["other_kernels_ms_per_step"], 4)},
    }
    if not args.headline_only:
        c2 = synth.C2_DISC
        log(f"gas disc {c2.name}, FP64")
        r2 = timed_rate(rossbi, torch, c2, rossbi.RB_FP64, 100, 5)
        r2["steps"] = 100
        out["gas_disc_fp64"] = {"workload": c2.name, "zone_updates_per_s": r2["zone_updates_per_s"],
                                "ms_per_step": round(r2["ms_per_step"], 4),
                                "roofline": kernel_roofline(c2, False, r2),
                                "step_hbm": step_hbm(c2, False, r2["ms_per_step"])}
        if not args.no_forms:
            out["precision_forms"] = precision_forms(rossbi, torch, args.forms_steps)
        if not args.no_adjoint:
            out["adjoint"] = adjoint_cost(rossbi, torch, args.adjoint_steps, 20)
        if not args.no_extensions:
            out["extensions"] = extensions(rossbi, torch, args.extensions_steps)
        if not args.no_cpu:
            log("cpu baseline (oracle)")
            out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
