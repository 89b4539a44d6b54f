"""Pins of the oracle's object mapping, boundary links and flag changes
(Sec. 2.3) against brute force and bookkeeping identities."""
import copy
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle import OracleSim, coupling, lbm
from oracle.d3q19 import E, OPP, Q, W as WT


def _brute_inside(body, p, dims, periodic):
    # independent formulation: a capsule is a cylinder plus two end balls
    X = np.array(body["X"], dtype=float)
    d = np.array(p) - X
    for k in range(3):
        if periodic[k]:
            L = dims[k]
            d[k] -= L * round(d[k] / L)
    r = body["radius"]
    if body["shape"] == coupling.SPHERE:
        return float(d @ d), r * r
    a = np.array([float(v) for v in coupling.quat_axis(body["quat"])])
    h = body["half_len"]
    t = float(d @ a)
    perp = d - t * a
    cands = [float((d - h * a) @ (d - h * a)), float((d + h * a) @ (d + h * a))]
    if abs(t) <= h:
        cands.append(float(perp @ perp))
    return min(cands), r * r


@pytest.mark.parametrize("seed", range(6))
def test_map_matches_brute_force(seed):
    case = W.random_small(seed)
    sim = OracleSim(case)
    nx, ny, nz = sim.dims
    for c in range(sim.N):
        i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
        want = 0
        for b, body in enumerate(sim.bodies):
            d2, r2 = _brute_inside(body, (i + 0.5, j + 0.5, k + 0.5), sim.dims, sim.periodic)
            if abs(d2 - r2) < 1e-9:
                want = -1  # tie within rounding: either answer is admissible
                break
            if d2 <= r2:
                want = 1 + b
                break
        if want >= 0:
            assert sim.flags[c] == want, (c, want, sim.flags[c])


@pytest.mark.parametrize("seed", range(3))
def test_links_match_brute_force(seed):
    case = W.random_small(seed)
    sim = OracleSim(case)
    nx, ny, nz = sim.dims
    n = (nx, ny, nz)
    want = []
    for c in range(sim.N):
        if sim.flags[c]:
            continue
        x = (c % nx, (c // nx) % ny, c // (nx * ny))
        for a in range(1, Q):
            y = [x[d] + E[a, d] for d in range(3)]
            if any((not sim.periodic[d]) and not (0 <= y[d] < n[d]) for d in range(3)):
                continue
            y = [y[d] % n[d] for d in range(3)]
            yc = y[0] + nx * (y[1] + ny * y[2])
            if sim.flags[yc]:
                want.append((c, a, int(sim.flags[yc]) - 1))
    got = list(zip(*[v.tolist() for v in sim.links]))
    assert got == sorted(want)


@pytest.mark.parametrize("r,cells,nlinks", [(3, 136, 696), (4, 280, 1176), (5, 552, 1896),
                                            (6, 912, 2592)])
def test_sphere_cell_and_link_counts(r, cells, nlinks):
    # integer-centred spheres: counts from direct enumeration of half-integer
    # points (x^2 + y^2 + z^2 <= r^2) and of their outward D3Q19 links
    pts = {p for p in itertools.product(np.arange(-r, r) + 0.5, repeat=3)
           if p[0] ** 2 + p[1] ** 2 + p[2] ** 2 <= r * r}
    assert len(pts) == cells
    out = sum(1 for p in pts for e in E[1:] if tuple(np.add(p, e)) not in pts)
    assert out == nlinks
    L = 2 * r + 6
    body = W.make_body(W.SPHERE, r, 1.0, (L / 2, L / 2, L / 2))
    sim = OracleSim(W.Case("s", L, L, L, 1.0, periodic=(True, True, True), bodies=[body]))
    assert int((sim.flags > 0).sum()) == cells
    assert len(sim.links[0]) == nlinks


def test_capsule_cell_and_link_counts():
    # capsule r = 5 with a cylinder of length 10 along x, centred on a lattice point
    body = W.make_body(W.CAPSULE, 5.0, 1.0, (20.0, 12.0, 12.0), h=5.0)
    sim = OracleSim(W.Case("c", 40, 24, 24, 1.0, periodic=(True, False, False), bodies=[body]))
    pts = set()
    for p in itertools.product(np.arange(10, 30) + 0.5, np.arange(7, 17) + 0.5, np.arange(7, 17) + 0.5):
        x = p[0] - 20.0
        t = min(max(x, -5.0), 5.0)
        if (x - t) ** 2 + (p[1] - 12) ** 2 + (p[2] - 12) ** 2 <= 25.0:
            pts.add(p)
    assert int((sim.flags > 0).sum()) == len(pts) == 1352
    assert len(sim.links[0]) == 3696


def test_refill_sets_equilibrium_at_object_velocity():
    # a cell uncovered by a moving sphere gets moments rho = mean neighbour
    # density and u = object velocity at the cell centre
    case = W.forced_motion(steps=0)
    df0 = W.initial_populations(case, seed=9, amp=1e-4)
    sim = OracleSim(case, df0=df0)
    found = 0
    for _ in range(25):
        before_flags = sim.flags.copy()
        before_df = sim.df.copy()
        bodies = copy.deepcopy(sim.bodies)
        sim.bodies = bodies
        new = coupling.map_bodies(bodies, sim.dims, sim.periodic)
        unc = np.nonzero((before_flags > 0) & (new == 0))[0]
        sim.step()
        if unc.size == 0:
            continue
        # recompute the refill on a copy and check its moments
        df = before_df.copy()
        coupling.refill(df, before_flags, new, sim.nbr, bodies, sim.dims, sim.periodic)
        for c in unc:
            rho = 1.0 + df[:, c].sum()
            u = (E.T @ df[:, c]) / rho
            uw = coupling.wall_velocity(bodies[0], np.array([c]), sim.dims, sim.periodic)
            assert np.allclose(u, [v[0] for v in uw], rtol=0, atol=1e-15)
            nb = [sim.nbr[a, c] for a in range(1, Q)]
            nb = [n for n in nb if n >= 0 and before_flags[n] == 0 and new[n] == 0]
            want = 1.0 + np.mean([before_df[:, n].sum() for n in nb])
            assert math.isclose(rho, want, rel_tol=0, abs_tol=1e-15)
            found += 1
    assert found > 5


def test_forced_motion_mass_bookkeeping():
    # every mass change comes from moving bounce-back, refilled cells and
    # dropped (covered) cells, exactly up to rounding
    case = W.forced_motion(steps=0)
    sim = OracleSim(case)
    events = 0
    for _ in range(30):
        m0 = math.fsum(sim.df.ravel())
        old_flags = sim.flags.copy()
        old_df = sim.df.copy()
        body = copy.deepcopy(sim.bodies[0])
        sim.step()
        new_flags = sim.flags
        unc = (old_flags > 0) & (new_flags == 0)
        cov = (old_flags == 0) & (new_flags > 0)
        events += int(unc.sum() + cov.sum())
        lc, ld, lb = sim.links
        y = sim.nbr[ld, lc]
        u = coupling.wall_velocity(body, y, sim.dims, sim.periodic)
        eo = E[OPP[ld]]
        eu = eo[:, 0] * u[0] + eo[:, 1] * u[1] + eo[:, 2] * u[2]
        bb = (6.0 * WT[ld] * sim.rho[lc] * eu).tolist()
        # refill mass enters before the sweep; covered mass leaves
        refill_df = old_df.copy()
        coupling.refill(refill_df, old_flags, new_flags, sim.nbr, [body], sim.dims, sim.periodic)
        gained = refill_df[:, unc].ravel().tolist()
        lost = old_df[:, cov].ravel().tolist()
        m1 = math.fsum(sim.df.ravel())
        want = math.fsum(bb + gained + [-v for v in lost])
        assert abs((m1 - m0) - want) < 1e-16 * sim.N
    assert events > 20
