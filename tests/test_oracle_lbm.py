"""Pins of the oracle's lattice part against closed forms and invariants
(D3Q19 tables, equilibrium moments, collision invariants, rest state, mass
and momentum bookkeeping)."""
import copy
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle import coupling, lbm
from oracle.d3q19 import E, OPP, Q, W as WT
from oracle.sim import OracleSim


def test_velocity_set_isotropy():
    # D3Q19 lattice tensors (Sec. 2.1): sum w = 1, sum w e = 0,
    # sum w e e = I/3, sum w e e e = 0, sum w e e e e = (d d + d d + d d)/9
    assert math.isclose(WT.sum(), 1.0, rel_tol=0, abs_tol=1e-15)
    assert np.allclose(WT @ E, 0.0, atol=1e-16)
    for a, b in itertools.product(range(3), repeat=2):
        m2 = np.sum(WT * E[:, a] * E[:, b])
        assert math.isclose(m2, (a == b) / 3.0, abs_tol=1e-15)
    for a, b, c in itertools.product(range(3), repeat=3):
        assert abs(np.sum(WT * E[:, a] * E[:, b] * E[:, c])) < 1e-16
    for a, b, c, d in itertools.product(range(3), repeat=4):
        m4 = np.sum(WT * E[:, a] * E[:, b] * E[:, c] * E[:, d])
        want = ((a == b) * (c == d) + (a == c) * (b == d) + (a == d) * (b == c)) / 9.0
        assert math.isclose(m4, want, abs_tol=1e-15)
    # 19 distinct velocities: rest, 6 axis, 12 face diagonals
    assert len({tuple(e) for e in E}) == 19
    assert sorted(int(v) for v in (E * E).sum(1)) == [0] + [1] * 6 + [2] * 12
    assert np.array_equal(E[OPP], -E)
    assert np.array_equal(OPP[OPP], np.arange(Q))


def test_equilibrium_moments():
    # f_eq reproduces rho, rho u and the Euler stress rho u u + rho I/3
    rng = np.random.default_rng(0)
    rho = 1.0 + 0.05 * rng.standard_normal(50)
    u = [0.05 * rng.standard_normal(50) for _ in range(3)]
    feq = lbm.equilibrium_dev(rho - 1.0, u) + WT[:, None]
    assert np.allclose(feq.sum(0), rho, rtol=0, atol=1e-15)
    for a in range(3):
        assert np.allclose(E[:, a] @ feq, rho * u[a], rtol=0, atol=1e-15)
        for b in range(3):
            pi = np.einsum("q,q...->...", E[:, a] * E[:, b], feq)
            assert np.allclose(pi, rho * u[a] * u[b] + rho * (a == b) / 3.0, atol=1e-15)


@pytest.mark.parametrize("tau", [0.51, 0.8, 1.0, 1.7])
def test_collision_conserves_mass_and_momentum(tau):
    rng = np.random.default_rng(1)
    df = 1e-3 * rng.standard_normal((19, 200))
    dft, rho, u = lbm.collide(df, tau)
    assert np.allclose(dft.sum(0), df.sum(0), rtol=0, atol=2e-17)
    assert np.allclose(E.T @ dft, E.T @ df, rtol=0, atol=2e-17)
    # moments of the non-conserved part relax by (1 - 1/tau)
    if tau == 1.0:
        assert np.allclose(dft, lbm.equilibrium_dev(rho - 1.0, u), atol=1e-18)


def test_collision_relaxes_stress_by_one_minus_omega():
    # the non-equilibrium stress is multiplied by (1 - 1/tau) (single relaxation time)
    rng = np.random.default_rng(2)
    df = 1e-3 * rng.standard_normal((19, 64))
    tau = 0.73
    dft, rho, u = lbm.collide(df, tau)
    feq = lbm.equilibrium_dev(rho - 1.0, u)
    for a, b in [(0, 0), (0, 1), (1, 2), (2, 2)]:
        c = E[:, a] * E[:, b]
        neq_before = c @ (df - feq)
        neq_after = c @ (dft - feq)
        assert np.allclose(neq_after, (1.0 - 1.0 / tau) * neq_before, atol=1e-16)


def test_streaming_is_a_permutation_in_a_periodic_box():
    # with no walls and no objects, streaming moves every population to the
    # neighbour cell: shifting back with numpy's roll recovers the input
    nx, ny, nz = 5, 4, 3
    nbr = lbm.neighbour_table(nx, ny, nz, (True, True, True))
    rng = np.random.default_rng(3)
    dft = rng.standard_normal((19, nx * ny * nz))
    flags = np.zeros(nx * ny * nz, dtype=np.uint8)
    out = lbm.stream_bounce_back(dft, 1.0 + dft.sum(0), flags, nbr, None)
    for a in range(19):
        f = dft[a].reshape(nz, ny, nx)
        want = np.roll(f, shift=(E[a, 2], E[a, 1], E[a, 0]), axis=(0, 1, 2))
        assert np.array_equal(out[a].reshape(nz, ny, nx), want)


def test_wall_bounce_back_reverses_momentum_at_walls():
    # a single population next to a wall comes back in the opposite direction
    nx, ny, nz = 3, 3, 3
    nbr = lbm.neighbour_table(nx, ny, nz, (True, False, False))
    dft = np.zeros((19, 27))
    c = 1 + nx * (2 + ny * 1)  # (1, 2, 1): touches the y = ny wall
    dft[3, c] = 0.25  # +y
    out = lbm.stream_bounce_back(dft, np.ones(27), np.zeros(27, np.uint8), nbr, None)
    assert out[4, c] == 0.25 and np.count_nonzero(out) == 1


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.9])
def test_rest_state_is_exactly_fixed(tau):
    # dF = 0 with objects at rest stays bit-exactly zero (rest weights cancel)
    case = W.plain_f64_small()
    case.tau = tau
    case.drives = []
    sim = OracleSim(case)
    sim.run(5)
    assert not np.any(sim.df)
    assert all(not np.any(np.asarray(F)) for F in sim.F)


def _static_case():
    case = W.plain_f64_small()
    case.drives = []
    case.springs = []
    for b in case.bodies:
        b.kinematic = True
    return case


def test_mass_conserved_with_static_objects():
    case = _static_case()
    df0 = W.initial_populations(case, seed=4, amp=1e-4)
    sim = OracleSim(case, df0=df0)
    m0 = math.fsum(sim.df.ravel())
    for _ in range(10):
        sim.step()
    m1 = math.fsum(sim.df.ravel())
    assert abs(m1 - m0) < 1e-15 * sim.N


def _momentum(df):
    return np.array([math.fsum((E[:, d] @ df).tolist()) for d in range(3)])


def _wall_links_force(sim, dft):
    # sum of e_alpha 2 dF~_alpha over links that leave through a wall
    fluid = np.nonzero(sim.flags == 0)[0]
    tot = np.zeros(3)
    for a in range(1, Q):
        wall = fluid[sim.nbr[a, fluid] < 0]
        tot += 2.0 * E[a] * math.fsum(dft[a, wall].tolist())
    return tot


@pytest.mark.parametrize("moving", [False, True])
def test_per_step_momentum_balance(moving):
    # fluid momentum change = -(sum of object forces minus their geometric
    # part) - wall exchange, exact up to rounding in a step without flag changes
    case = W.plain_f64_small()
    if moving:
        for i, b in enumerate(case.bodies):
            b.vel = (1e-3 * (i + 1), -2e-4, 3e-4)
            b.omega = (1e-4, 2e-4 * i, -1e-4)
    df0 = W.initial_populations(case, seed=5, amp=1e-4)
    sim = OracleSim(case, df0=df0)
    for _ in range(3):
        p0 = _momentum(sim.df)
        m0 = math.fsum(sim.df.ravel())
        before = copy.deepcopy(sim.bodies)  # u_w of step n uses the state at n
        sim.step()
        assert sim.last_changes == (0, 0)
        p1 = _momentum(sim.df)
        m1 = math.fsum(sim.df.ravel())
        # geometric part of the force: integer sum / 36
        lc, ld, lb = sim.links
        Fdev = np.zeros(3)
        dmass = []
        for b in range(len(sim.bodies)):
            sel = lb == b
            G = (E[ld[sel]] * np.where(ld[sel] <= 6, 4, 2)[:, None]).sum(0) / 36.0
            Fdev += np.array(sim.F[b]) - G
            y = sim.nbr[ld[sel], lc[sel]]
            u = coupling.wall_velocity(before[b], y, sim.dims, sim.periodic)
            eo = E[OPP[ld[sel]]]
            eu = eo[:, 0] * u[0] + eo[:, 1] * u[1] + eo[:, 2] * u[2]
            dmass.extend((6.0 * WT[ld[sel]] * sim.rho[lc[sel]] * eu).tolist())
        fw = _wall_links_force(sim, sim.dft)
        scale = 1e-4 * len(lc)
        assert np.allclose(p1 - p0, -(Fdev + fw), rtol=0, atol=1e-13 * scale)
        assert abs((m1 - m0) - math.fsum(dmass)) < 1e-13 * scale


def test_mirror_symmetry_gives_no_transverse_force():
    # the swimmer setup is mirror-symmetric in y and z: F_y, F_z and T vanish
    sim = OracleSim(W.plain_f64_small())
    sim.run(30)
    for b in range(3):
        F = np.abs(np.array(sim.F[b]))
        T = np.abs(np.array(sim.T[b]))
        assert F[0] > 1e-6
        assert F[1] < 1e-18 and F[2] < 1e-18
        assert np.all(T < 1e-17)
