"""Launch-shape autotuner for the sweep and the step sequence.

For a key (box shapes, storage type) it times every candidate tuning of
``CANDIDATES`` on a short run of the caller's own context and keeps the
fastest; results are cached as JSON (default ``~/.cache/lbmswim/tuning.json``,
override with ``LBMSWIM_TUNING_CACHE``).  Every candidate produces bitwise
identical results (fixed-order reductions), so tuning never changes numbers.
"""
from __future__ import annotations

import json
import os
import time

CANDIDATES = [
    {"block": b, "xcd_order": x, "graph_steps": g}
    for b in (128, 256, 512) for x in (0, 1) for g in (16, 64)
]


def cache_path():
    return os.environ.get("LBMSWIM_TUNING_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "lbmswim", "tuning.json"))


def key_of(sim):
    shapes = sorted({(b.case.nx, b.case.ny, b.case.nz) for b in sim.boxes})
    return f"{sim.storage}|{len(sim.boxes)}|" + ";".join("x".join(map(str, s)) for s in shapes)


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(table):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def timed_steps(steps, graph_steps):
    """Steps of a candidate's timing run: ``steps`` rounded up to a whole,
    non-zero number of its graphs (lbm_step replays a graph only for runs of
    at least ``graph_steps`` steps, and launches the remainder one by one)."""
    if graph_steps <= 0:
        return max(steps, 1)
    return graph_steps * max(1, -(-steps // graph_steps))


def tune(sim, steps=64, use_cache=True, verbose=False):
    """Pick and apply the fastest candidate for ``sim`` (a Sim or BatchSim).

    The timing run advances the simulation; callers that need an untouched
    state tune a scratch context of the same shapes.  Returns the chosen
    tuning dict."""
    import torch

    table = _load() if use_cache else {}
    key = key_of(sim)
    if key in table:
        best = table[key]["tuning"]
        for k, v in best.items():
            sim.tune(k, v)
        return best
    results = []
    for cand in CANDIDATES:
        for k, v in cand.items():
            sim.tune(k, v)
        g = cand["graph_steps"]
        sim.step(g)  # capture and warm up
        torch.cuda.synchronize()
        # a whole number of graphs, at least one: a shorter run would launch
        # every kernel itself and time another launch sequence
        n = timed_steps(steps, g)
        t0 = time.perf_counter()
        sim.step(n)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / n
        results.append((dt, cand))
        if verbose:
            print(f"[autotune] {key} {cand}: {dt * 1e6:.1f} us/step", flush=True)
    dt, best = min(results, key=lambda r: r[0])
    for k, v in best.items():
        sim.tune(k, v)
    table[key] = {"tuning": best, "us_per_step": dt * 1e6}
    if use_cache:
        _store(table)
    return best
