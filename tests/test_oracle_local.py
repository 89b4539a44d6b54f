"""The cell-by-cell step of oracle.local agrees with the full-grid oracle
step (same rules in pull form) on a box with walls, bodies and a moving
kinematic body."""
import numpy as np

import workloads as W
from oracle import OracleSim, local


def test_step_at_matches_full_step():
    case = W.random_small(2)
    df0 = W.initial_populations(case, seed=3, amp=1e-3)
    sim = OracleSim(case, df0=df0).run(3).map_next()
    flags = sim.flags.copy()
    known = local.Known(np.arange(sim.N), sim.df.copy())
    bodies = [dict(b) for b in sim.bodies]
    lc, ld, lb = local.links_at(np.arange(sim.N), flags, sim.dims, sim.periodic)
    assert all(np.array_equal(x, y) for x, y in zip((lc, ld, lb), sim.links))
    F, T = local.forces_at(known, lc, ld, lb, bodies, sim.dims, sim.periodic, case.tau)
    fluid = np.nonzero(flags == 0)[0]
    got = local.step_at(known, fluid, flags, bodies, sim.dims, sim.periodic, case.tau)
    sim.step()
    assert np.array_equal(got, sim.df[:, fluid])
    assert np.allclose(np.array(F), np.array(sim.F), rtol=0, atol=0)
    assert np.allclose(np.array(T), np.array(sim.T), rtol=0, atol=0)
