"""Oracle runs for the GPU parity tests, in worker processes (spawned, so
that they never inherit a GPU context): each job runs one workload with the
CPU oracle and returns its per-step trajectory and final state."""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def run_case(case, steps):
    """(F, T, D, V) per step as arrays (steps, bodies, 3), the deviations after
    the next mapping (19, nz, ny, nx) and the flags after it."""
    from oracle import OracleSim
    sim = OracleSim(case).run(steps)
    F = np.array([t["F"] for t in sim.traj], dtype=float)
    T = np.array([t["T"] for t in sim.traj], dtype=float)
    D = np.array([t["D"] for t in sim.traj], dtype=float)
    V = np.array([t["V"] for t in sim.traj], dtype=float)
    sim.map_next()
    return F, T, D, V, sim.populations().copy(), sim.flags.copy()


def run_many(jobs, workers=4):
    """Run [(case, steps), ...] in parallel worker processes, results in order."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=min(workers, len(jobs)), mp_context=mp.get_context("spawn")) as ex:
        futs = [ex.submit(run_case, c, s) for c, s in jobs]
        return [f.result() for f in futs]
