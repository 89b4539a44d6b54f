"""Parity at the full workload sizes (256x128x128 and 512x256x256), in the
launch configuration the benchmark times: flags and boundary links are
checked bit for bit around the bodies (and the rest of the box must be plain
fluid); one coupled step is checked at a seeded sample of cells plus every
boundary cell against the oracle's cell-by-cell step from the same state,
and the body forces against the oracle's momentum exchange."""
import numpy as np
import pytest

import workloads as W
from oracle import coupling, local

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-6, "f16s": 2e-3, "bf16s": 1.6e-2}


def _oracle_bodies(gpu_bodies, case):
    out = []
    for g, c in zip(gpu_bodies, case.bodies):
        b = {"shape": c.shape, "radius": c.radius, "half_len": c.half_len, "anchor": list(c.anchor),
             "D": list(g["D"]), "quat": list(g["quat"]), "V": list(g["V"]), "Omega": list(g["Omega"])}
        b["X"] = [b["anchor"][k] + b["D"][k] for k in range(3)]
        out.append(b)
    return out


def _region(case, bodies):
    # cells within the bounding box of every body, plus 3 cells
    nx, ny, nz = case.nx, case.ny, case.nz
    cells = []
    for b in bodies:
        e = b["radius"] + b["half_len"] + 3
        rng = [np.arange(int(np.floor(b["X"][k] - e)), int(np.floor(b["X"][k] + e)) + 1) for k in range(3)]
        rng = [r % n if case.periodic[k] else r[(r >= 0) & (r < n)] for k, (r, n) in enumerate(zip(rng, (nx, ny, nz)))]
        k, j, i = np.meshgrid(rng[2], rng[1], rng[0], indexing="ij")
        cells.append((i + nx * (j + ny * k)).ravel())
    return np.unique(np.concatenate(cells))


@pytest.mark.parametrize("name,storage", [("plain", "f32"), ("plain", "f64"), ("plain", "f16s"),
                                          ("capsule_SCS", "f32"), ("capsule_CCC", "f32"),
                                          ("capsule_SCS", "bf16s")])
def test_full_size_sampled_step(name, storage):
    from paper_1108_0786_amd.sim import Sim
    case = W.plain_at_scale(storage=storage) if name == "plain" else W.capsule_full(name.split("_")[1], storage)
    print(f"[gpu] full size {case.name} {storage}", flush=True)
    sim = Sim(case, storage=storage)
    sim.step(3)
    dims, per = (case.nx, case.ny, case.nz), case.periodic
    flags_gpu = sim.flags()
    owner = (flags_gpu & 0x7F).astype(np.int64)
    bodies = _oracle_bodies(sim.bodies(), case)
    # flags and links, bit for bit, around the bodies; plain fluid elsewhere
    region = _region(case, bodies)
    want = np.zeros(region.size, dtype=np.int64)
    for b in reversed(range(len(bodies))):
        r = coupling.lever_arms(bodies[b]["X"], region, dims, per)
        want[coupling.inside(bodies[b], r)] = b + 1
    assert np.array_equal(owner[region], want)
    outside = np.ones(case.ncells, dtype=bool)
    outside[region] = False
    assert not np.any(flags_gpu[outside])
    lc, ld, lb = local.links_at(region, owner, dims, per)
    g = sim.links()
    assert all(np.array_equal(x, y) for x, y in zip(g, (lc, ld, lb)))
    near = np.zeros(case.ncells, dtype=bool)
    near[lc] = True
    assert np.array_equal((flags_gpu & 0x80) != 0, near)
    # one step at a sample of cells: random fluid cells, all boundary cells, wall rows
    rng = np.random.default_rng(2024)
    fluid = np.nonzero(owner == 0)[0]
    sample = np.unique(np.concatenate([rng.choice(fluid, 20000, replace=False), lc,
                                       rng.choice(fluid[(fluid // case.nx) % case.ny == 0], 2000)]))
    need = local.neighbours(sample, dims, per, sign=-1)
    src = np.unique(np.concatenate([sample, need[need >= 0]]))
    known = local.Known(src, sim.populations_at(src))
    F_orc, T_orc = local.forces_at(known, lc, ld, lb, bodies, dims, per, case.tau)
    want_df = local.step_at(known, sample, owner, bodies, dims, per, case.tau)
    sim.step(1)
    got = sim.populations_at(sample)
    F, T = sim.forces()
    err = np.abs(got - want_df).max() / np.abs(want_df).max()
    errF = np.abs(F - np.array(F_orc)).max() / np.abs(np.array(F_orc)).max()
    print(f"[gpu] full size {case.name} {storage}: {sample.size} cells, {lc.size} links, "
          f"dF err {err:.2e}, F err {errF:.2e}", flush=True)
    assert err < TOL[storage]
    assert errF < max(TOL[storage], 1e-12)
    sim.close()
