"""Throughput of the coupled swimmer step on one MI355X.

Workload: one three-sphere swimmer (r = 6, rest length 24, amplitude drawn
with seed 0) in a 256x128x128 channel, tau = 0.8 (periodic x, walls y and
z), populations stored as FP32 deviations; further legs time the same
workload with FP64, shifted-FP16 and shifted-BF16 storage.  A step is one
full coupled step: sweep (collide, stream, bounce-back, link records) plus
the coupling kernel (momentum exchange, driving, springs, integration,
mapping check).  FP32 streams in place (one population buffer, its layout
alternating with the step's parity); the other storages push into a second
buffer (the library's defaults).  Inputs are resident in HBM before timing
starts.

Prints one JSON line.  ``value`` is MLUPS (lattice-cell updates per second
over the whole box, / 1e6) of the FP32 leg; ``roofline`` divides the
sweep kernel's algorithmic bytes per launch by its mean launch time taken
from HIP events recorded on the library's stream around every sweep of a
second pass of the same number of steps (launched one by one, since the
events cannot sit inside the replayed graphs), and sets that rate beside
two measured ceilings: a plain streaming copy and a copy with the
two-buffer sweep's access pattern (``lbm_stream_copy``); ``cpu_baseline``
times the CPU oracle on a few steps of the same box."""
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

# HBM bytes per launch of the default FP32 sweep (in place) at 256x128x128,
# the mean of even and odd steps, from two rocprofv3 counter passes
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0; the factors make the counters read
# 2 GiB for a 2 GiB copy).  Valid only for the kernel sources whose digest is
# given; a changed kernel reports null until it is measured again.
SWEEP_TRAFFIC = {"bytes": 660199441,
                 "sources": ("common.h", "geometry.h", "sweep.h", "sweep_aa.h"),
                 "sha256": "bfc485eb76f9907b0c58fd9a7e9bc06cb59e170cf93102c94c3ba22f00512873"}


def measured_traffic():
    import hashlib
    h = hashlib.sha256()
    for name in SWEEP_TRAFFIC["sources"]:
        with open(os.path.join(ROOT, "paper_1108_0786_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return SWEEP_TRAFFIC["bytes"] if h.hexdigest() == SWEEP_TRAFFIC["sha256"] else None


def sweep_bytes(case, n_fluid, storage):
    """Algorithmic HBM bytes of one sweep launch: every fluid cell reads and
    writes its 19 populations; every cell's flag byte is read once."""
    s = STORAGE_BYTES[storage]
    return n_fluid * 2 * 19 * s + case.ncells


def time_leg(case, storage, steps, warmup, tune=None):
    import numpy as np
    import torch

    from paper_1108_0786_amd.sim import Sim

    print(f"[bench] leg {storage}: {case.name}, warmup {warmup}, steps {steps}", file=sys.stderr, flush=True)
    sim = Sim(case, storage=storage, device="cuda:0", shift_log2=16, tune=tune)
    n_fluid = int((sim.flags() & 0x7F == 0).sum())
    sim.step(warmup)
    # capture the graphs the timed run replays (nothing runs)
    sim.prepare(steps)
    torch.cuda.synchronize()
    # throughput: steps replayed from HIP graphs, nothing recorded in between
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.status()
    # kernel durations: the same number of steps again, launched one by one with
    # HIP events recorded around every sweep and coupling launch on the
    # library's stream
    sim.set_timing(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
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
        "ms_per_step_timed_launches": (t3 - t2) / steps * 1e3,
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


def batched_leg(periods=10):
    """Parameter sweep: 96 swimmers in their own boxes (seed 7), each advanced
    10 periods (4000-12000 steps), once as one batched context (one launch per
    kernel per step for all active boxes, replayed from HIP graphs, launch
    shapes from the autotuner) and once box after box."""
    import torch

    import workloads as W
    from paper_1108_0786_amd import autotune
    from paper_1108_0786_amd.sim import BatchSim, Sim

    cases = W.batched_sweep(seed=7, periods=periods, storage="f32")
    lups = sum(c.ncells * c.steps for c in cases)
    print(f"[bench] batched sweep: {len(cases)} boxes, {sum(c.ncells for c in cases)} cells, "
          f"{lups:.3e} cell updates", file=sys.stderr, flush=True)
    scratch = BatchSim(cases, storage="f32")
    best = autotune.tune(scratch, steps=32)
    scratch.close()
    del scratch
    batch = BatchSim(cases, storage="f32", tune=best)
    for b, c in enumerate(cases):
        batch.set_step_limit(b, c.steps)
    batch.prepare(max(c.steps for c in cases))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(max(c.steps for c in cases))
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    batch.status()
    disp = [batch.bodies(b)[0]["D"][0] for b in range(len(cases))]
    batch.close()
    del batch
    print(f"[bench] batched: {t_batch:.2f} s ({lups / t_batch / 1e6:.0f} MLUPS), tuning {best}",
          file=sys.stderr, flush=True)
    t_seq = 0.0
    for i, c in enumerate(cases):
        sim = Sim(c, storage="f32")
        sim.prepare(c.steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(c.steps)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        same = sim.bodies()[0]["D"][0] == disp[i]
        assert same, f"batched and sequential runs differ for {c.name}"
        sim.close()
    print(f"[bench] sequential: {t_seq:.2f} s ({lups / t_seq / 1e6:.0f} MLUPS)", file=sys.stderr, flush=True)
    return {"boxes": len(cases), "cell_updates": lups, "batched_s": round(t_batch, 3),
            "sequential_s": round(t_seq, 3), "batched_mlups": round(lups / t_batch / 1e6, 1),
            "sequential_mlups": round(lups / t_seq / 1e6, 1), "speedup": round(t_seq / t_batch, 3),
            "tuning": best, "bitwise_equal_middle_body_displacement": True}


def adjoint_leg(steps=1000, every=50):
    """The hand-written reverse pass on the 128x64x64 adjoint workload (FP64,
    tau 0.9, r = 4 swimmer, two periods of 500 steps): wall time of
    ``lbm_adjoint`` over ``steps`` steps with checkpoints every ``every``,
    beside the same number of forward steps replayed from graphs.  The
    reverse pass runs every step forward twice (once to take checkpoints,
    once per segment to rebuild its states) and one adjoint sweep
    (``adjoint_sweep_kernel``) per step."""
    import torch

    import workloads as W
    from paper_1108_0786_amd.sim import Sim

    case = W.adjoint_case(storage="f64", periods=steps // 500)
    print(f"[bench] adjoint: {case.name}, {steps} steps, checkpoints every {every}", file=sys.stderr, flush=True)
    fwd = Sim(case, storage="f64", device="cuda:0")
    n_fluid = int((fwd.flags() & 0x7F == 0).sum())
    fwd.prepare(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fwd.step(steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    fwd.close()
    adj = Sim(case, storage="f64", device="cuda:0")
    adj.adjoint(steps // 10, every)          # first call: scratch allocation and kernel loading
    adj.close()
    adj = Sim(case, storage="f64", device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, grad = adj.adjoint(steps, every)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    adj.close()
    # adjoint sweep per fluid cell: the forward deviations (19 doubles) and
    # the adjoint of the next step (19 doubles) in, the adjoint out (19
    # doubles), and the flag byte
    per_cell = 19 * 8 * 3 + 1
    out = {"workload": f"{case.nx}x{case.ny}x{case.nz} FP64 swimmer, tau {case.tau}", "steps": steps,
           "checkpoint_every": every, "forward_s": round(t_fwd, 4), "adjoint_s": round(t_adj, 4),
           "ratio": round(t_adj / t_fwd, 2), "adjoint_sweep_bytes_per_fluid_cell": per_cell,
           "fluid_cells": n_fluid, "J": J, "grad": [float(g) for g in grad]}
    print(f"[bench] adjoint: forward {t_fwd * 1e3:.1f} ms, adjoint {t_adj * 1e3:.1f} ms "
          f"({t_adj / t_fwd:.1f}x)", file=sys.stderr, flush=True)
    return out


def copy_ceiling(nbytes=2 << 30, reps=20):
    """Practical HBM ceiling: the best of a few launch shapes of a plain
    streaming copy of ``nbytes`` (read + write counted), timed with torch
    events on the stream it runs on."""
    import ctypes as C

    import torch

    from paper_1108_0786_amd import _abi

    lib = _abi.load()
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream().cuda_stream
    best = 0.0
    for per_cu in (0, 32, 256):
        for nt in (0, 1):
            def run():
                rc = lib.lbm_copy_kernel(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes, per_cu,
                                         nt, C.c_void_p(stream))
                assert rc == 0
            for _ in range(3):
                run()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                run()
            b.record()
            torch.cuda.synchronize()
            gbs = 2 * nbytes / (a.elapsed_time(b) / reps / 1e3) / 1e9
            shape = "one vector per thread" if per_cu == 0 else f"{per_cu} blocks/CU"
            print(f"[bench] copy {shape} nontemporal={nt}: {gbs:.0f} GB/s", file=sys.stderr, flush=True)
            best = max(best, gbs)
    del src, dst
    return best


def pattern_ceiling(n, stride, elem_bytes, reps=20):
    """Practical ceiling of the sweep's access pattern at this box size: the
    best of plain and non-temporal loads for ``lbm_stream_copy`` (19 streams
    of ``n`` elements in, 19 out, the sweep's stride), read + write counted,
    timed with torch events on the stream it runs on."""
    import ctypes as C

    import torch

    from paper_1108_0786_amd import _abi

    lib = _abi.load()
    nbytes = 19 * stride * elem_bytes
    src = torch.ones(nbytes // 2, dtype=torch.int16, device="cuda:0")
    dst = torch.zeros_like(src)
    stream = torch.cuda.current_stream().cuda_stream
    best = 0.0
    for nt in (0, 1):
        def run():
            rc = lib.lbm_stream_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), n, stride,
                                     elem_bytes, nt, C.c_void_p(stream))
            assert rc == 0
        for _ in range(3):
            run()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            run()
        b.record()
        torch.cuda.synchronize()
        gbs = 2 * 19 * n * elem_bytes / (a.elapsed_time(b) / reps / 1e3) / 1e9
        print(f"[bench] sweep-pattern copy, {elem_bytes}-byte elements, nontemporal loads={nt}: {gbs:.0f} GB/s",
              file=sys.stderr, flush=True)
        best = max(best, gbs)
    del src, dst
    return best


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or the platform's."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def time_oracle(case, steps):
    from oracle import OracleSim

    sim = OracleSim(case)
    t0 = time.perf_counter()
    sim.run(steps)
    return case.ncells * steps / (time.perf_counter() - t0) / 1e6


def cpu_baseline(case, steps=8):
    """The oracle as it stands, on a bounded sample of the same box: NumPy
    elementwise kernels, one host core (no BLAS calls on this path)."""
    print(f"[bench] cpu baseline: oracle, {steps} steps of {case.name}", file=sys.stderr, flush=True)
    mlups = time_oracle(case, steps)
    return {"value": mlups, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{steps} coupled steps of the {case.nx}x{case.ny}x{case.nz} FP64 case on one host core",
            "cpu": cpu_model(), "cpus_visible": os.cpu_count()}


def cpu_configs():
    """The oracle on the other workloads (``--cpu-configs``): the 48x32x32
    case in full (400 steps), and 100-step samples of the 128x64x64 capsule
    crop and of the 128x64x64 adjoint workload, one host core each."""
    import workloads as W

    out = {}
    for name, case, steps in (("48x32x32, 400 steps", W.plain_f64_small(), 400),
                              ("capsule crop 128x64x64 S-C-S, 100 of 1000 steps", W.capsule_crop("SCS", "f64"), 100),
                              ("adjoint workload 128x64x64, 100 of 1000 steps", W.adjoint_case(storage="f64"), 100)):
        print(f"[bench] cpu: oracle, {name}", file=sys.stderr, flush=True)
        out[name] = round(time_oracle(case, steps), 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--legs", default="f32,f64,f16s,bf16s")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-periods", type=int, default=10)
    ap.add_argument("--streaming", choices=("default", "0", "1"), default="default",
                    help="population streaming of every leg: the library's default per storage, "
                         "0 two buffers, 1 in place")
    ap.add_argument("--adjoint", action="store_true",
                    help="also time the reverse pass on the 128x64x64 adjoint workload")
    ap.add_argument("--cpu-configs", action="store_true",
                    help="also time the oracle on the other workloads (several minutes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the swimmer step runs and is timed on a single "
              "MI355X; the slab decomposition over several GPUs is designed, not implemented", file=sys.stderr)
        sys.exit(2)

    import workloads as W

    legs = [s for s in args.legs.split(",") if s]
    if "f32" not in legs:
        legs = ["f32"] + legs
    results = {}
    tune = None if args.streaming == "default" else {"streaming": int(args.streaming)}
    for st in legs:
        results[st] = time_leg(W.plain_at_scale(storage=st), st, args.steps, args.warmup, tune=tune)
    head = results["f32"]
    case = W.plain_at_scale(storage="f32")
    copy_gbs = copy_ceiling()
    print(f"[bench] plain copy: {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)
    from paper_1108_0786_amd.sim import padded_stride
    for st, r in results.items():
        r["pattern_gbs"] = pattern_ceiling(case.ncells, padded_stride(case.ncells), STORAGE_BYTES[st])
        r["frac_of_pattern"] = r["sweep_gbs"] / r["pattern_gbs"]
    batched = None if args.no_batch else batched_leg(args.batch_periods)
    adjoint = adjoint_leg() if args.adjoint else None
    cpu = None if args.no_cpu else cpu_baseline(W.plain_at_scale(storage="f64"))
    if cpu is not None and args.cpu_configs:
        cpu["other_workloads_mlups"] = cpu_configs()
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
                     "unit": "GB/s", "frac": round(head["sweep_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic() if args.streaming == "default" else None,
                     "kernel": ("sweep_kernel<float> (two buffers)" if args.streaming == "0" else
                                "sweep_aa_kernel<float> (in-place streaming, mean of even and odd steps)"),
                     "bytes_per_launch": head["sweep_bytes"],
                     "launch_us": round(head["sweep_us"], 2), "copy_ceiling_gbs": round(copy_gbs, 1),
                     "frac_of_copy": round(head["sweep_gbs"] / copy_gbs, 4),
                     "two_buffer_pattern_ceiling_gbs": round(head["pattern_gbs"], 1),
                     "frac_of_two_buffer_pattern": round(head["frac_of_pattern"], 4)},
        "cpu_baseline": cpu,
        "batched_sweep": batched,
        "adjoint": adjoint,
        "legs": {k: {kk: (float(f"{vv:.6g}") if isinstance(vv, float) else vv) for kk, vv in v.items()}
                 for k, v in results.items()},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
