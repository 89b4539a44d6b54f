"""Throughput of the coupled swimmer step on one MI355X.

Workload: one three-sphere swimmer (r = 6, rest length 24, amplitude drawn
with seed 0) in a 256x128x128 channel, tau = 0.8 (periodic x, walls y and
z), populations stored as FP32 deviations; further legs time the same
workload with FP64, shifted-FP16 and shifted-BF16 storage.  A step is one
full coupled step: sweep (collide, stream, bounce-back, link records) plus
the coupling kernel (momentum exchange, driving, springs, integration,
mapping check).  Inputs are resident in HBM before timing starts.

Prints one JSON line.  ``value`` is MLUPS (lattice-cell updates per second
over the whole box, / 1e6) of the FP32 leg; ``roofline`` divides the
sweep kernel's algorithmic bytes per launch by its mean launch time taken
from HIP events recorded on the library's stream around every sweep of the
timed region; ``cpu_baseline`` times the CPU oracle on a few steps of the
same box."""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}


def sweep_bytes(case, n_fluid, storage):
    """Algorithmic HBM bytes of one sweep launch: every fluid cell reads and
    writes its 19 populations; every cell's flag byte is read once."""
    s = STORAGE_BYTES[storage]
    return n_fluid * 2 * 19 * s + case.ncells


def time_leg(case, storage, steps, warmup):
    import numpy as np
    import torch

    from paper_1108_0786_amd.sim import Sim

    print(f"[bench] leg {storage}: {case.name}, warmup {warmup}, steps {steps}", file=sys.stderr, flush=True)
    sim = Sim(case, storage=storage, device="cuda:0", shift_log2=16)
    n_fluid = int((sim.flags() & 0x7F == 0).sum())
    sim.step(warmup)
    torch.cuda.synchronize()
    sim.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sweep_ms, n_sweep, couple_ms, n_couple = sim.timing()
    sim.set_timing(False)
    sim.status()
    F, T = sim.forces()
    assert np.all(np.isfinite(F)), "non-finite forces"
    elapsed = t1 - t0
    sweep_avg_s = sweep_ms / 1e3 / max(n_sweep, 1)
    nbytes = sweep_bytes(case, n_fluid, storage)
    out = {
        "storage": storage,
        "mlups": case.ncells * steps / elapsed / 1e6,
        "mflups": n_fluid * steps / elapsed / 1e6,
        "ms_per_step": elapsed / steps * 1e3,
        "sweep_us": sweep_avg_s * 1e6,
        "couple_us": couple_ms / max(n_couple, 1) * 1e3,
        "sweep_gbs": nbytes / sweep_avg_s / 1e9,
        "sweep_bytes": nbytes,
        "displacement": sim.centroid_displacement(),
    }
    print(f"[bench] {storage}: {out['mlups']:.0f} MLUPS, sweep {out['sweep_us']:.1f} us "
          f"({out['sweep_gbs']:.0f} GB/s), coupling {out['couple_us']:.1f} us", file=sys.stderr, flush=True)
    sim.close()
    return out


def cpu_baseline(case, steps=3):
    """The oracle as it stands, on a few steps of the same box (single core:
    NumPy elementwise kernels)."""
    from oracle import OracleSim

    print(f"[bench] cpu baseline: oracle, {steps} steps of {case.name}", file=sys.stderr, flush=True)
    sim = OracleSim(case)
    t0 = time.perf_counter()
    sim.run(steps)
    t1 = time.perf_counter()
    return {"value": case.ncells * steps / (t1 - t0) / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{steps} coupled steps of the {case.nx}x{case.ny}x{case.nz} FP64 case on one host core"
                      f" ({platform.processor() or platform.machine()}, {os.cpu_count()} cpus visible)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--legs", default="f32,f64,f16s,bf16s")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the swimmer step is built and timed on a single "
              "MI355X (multi-GPU slab decomposition is a design, not part of this build)", file=sys.stderr)
        sys.exit(2)

    import workloads as W

    legs = [s for s in args.legs.split(",") if s]
    if "f32" not in legs:
        legs = ["f32"] + legs
    results = {}
    for st in legs:
        results[st] = time_leg(W.plain_at_scale(storage=st), st, args.steps, args.warmup)
    head = results["f32"]
    case = W.plain_at_scale(storage="f32")
    cpu = None if args.no_cpu else cpu_baseline(W.plain_at_scale(storage="f64"))
    line = {
        "metric": "MLUPS & % HBM roofline, fused D3Q19+moving-bead step, FP32 vs FP64/FP16, 1 GPU",
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"three-sphere swimmer, {case.nx}x{case.ny}x{case.nz} D3Q19 channel, tau 0.8, "
                               "r 6, rest length 24, FP32 shifted populations",
                   "cells": case.ncells, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(head["sweep_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(head["sweep_gbs"] / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "sweep_kernel<float>", "bytes_per_launch": head["sweep_bytes"],
                     "launch_us": round(head["sweep_us"], 2)},
        "cpu_baseline": cpu,
        "legs": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                 for k, v in results.items()},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
