"""Write the stored expected values that are too slow to recompute in a test.

Every value here comes from the CPU oracle alone (``oracle/``), on the seeded
workloads of ``workloads/``:

* ``capsule_crop_{SCS,CCC}.npz``: the capsule swimmers of the precision
  workload on the 128x64x64 crop, FP64, 1000 steps: per-step force, torque and
  displacement of the three bodies, and the final deviations at a seeded
  sample of 20000 cells.
* ``adjoint_tangent.json``: for the adjoint workload (128x64x64, two periods
  of 500 steps), the net x displacement J of the swimmer's centroid and its
  derivatives with respect to the driving amplitude, the phase lag and the
  spring stiffness, by the complex-step method (complex128 oracle run with an
  imaginary perturbation of 1e-20 times the parameter).

Usage: ``python tests/golden/make_goldens.py capsule SCS`` (or ``capsule
CCC``, ``adjoint value``, ``adjoint amplitude``, ``adjoint phase_lag``,
``adjoint k``); each job writes its own file so the jobs can run in parallel.
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import OracleSim  # noqa: E402


def capsule(design: str) -> None:
    case = W.capsule_crop(design, storage="f64")
    t0 = time.time()
    sim = OracleSim(case)
    for n in range(case.steps):
        sim.step()
        if n % 50 == 0:
            print(f"capsule {design}: step {n} ({time.time() - t0:.0f} s), "
                  f"max |F| {np.abs(np.array(sim.traj[-1]['F'])).max():.3e}", flush=True)
    sim.map_next()
    if not (np.all(np.isfinite(sim.df)) and all(np.all(np.isfinite(t["F"])) for t in sim.traj)):
        raise SystemExit(f"capsule {design}: the oracle run is not finite; nothing written")
    # the hydrodynamic forces of a stable run stay of the order of the driving
    Fmax = max(np.abs(np.array(t["F"])).max() for t in sim.traj)
    if Fmax > 20.0 * case.drives[0].amplitude:
        raise SystemExit(f"capsule {design}: max |F| {Fmax:.3e} is far above the driving; nothing written")
    F = np.array([t["F"] for t in sim.traj])
    T = np.array([t["T"] for t in sim.traj])
    D = np.array([t["D"] for t in sim.traj])
    rng = np.random.default_rng(12345)
    cells = np.sort(rng.choice(sim.N, size=20000, replace=False))
    np.savez_compressed(os.path.join(HERE, f"capsule_crop_{design}.npz"), F=F, T=T, D=D, cells=cells,
                        df=sim.df[:, cells], flags=sim.flags[cells], steps=case.steps)


def adjoint(which: str) -> None:
    case = W.adjoint_case(storage="f64")
    base = {"amplitude": case.drives[0].amplitude, "phase_lag": case.drives[0].phase_lag,
            "k": case.springs[0].k}
    t0 = time.time()
    if which == "value":
        sim = OracleSim(case)
        dtype_note = "float64"
    else:
        h = 1e-20 * base[which]
        sim = OracleSim(case, dtype=np.complex128, params={which: base[which] + 1j * h})
        dtype_note = f"complex128, h = 1e-20 * {which}"
    for n in range(case.steps):
        sim.step()
        if n % 50 == 0:
            print(f"adjoint {which}: step {n} ({time.time() - t0:.0f} s)", flush=True)
    J = sim.centroid_displacement()
    out = {"case": case.name, "steps": case.steps, "base": base, "run": dtype_note}
    if which == "value":
        out["J"] = float(J)
    else:
        out["J"] = float(np.real(J))
        out["dJ"] = float(np.imag(J) / (1e-20 * base[which]))
    with open(os.path.join(HERE, f"adjoint_tangent_{which}.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    kind, arg = sys.argv[1], sys.argv[2]
    {"capsule": capsule, "adjoint": adjoint}[kind](arg)
