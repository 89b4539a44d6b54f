"""Pins of the oracle's rotational coupling (Sec. 2.3: the object velocity
u_w = V + Omega x r enters the moving bounce-back; the torque is the sum of
the lever arm times the link term of Eq. hydroF; Alg. 1 advances Omega with
the torque).  Each test fixes one of these against something other than the
oracle itself:

* the angular-momentum balance of one step: the change of the fluid's
  angular momentum equals minus the torque that the momentum exchange hands
  to the bodies and to the walls (collision conserves momentum cell by
  cell, free streaming moves momentum along itself);
* the exact integer form of the geometric torque against a direct sum over
  the links;
* the integrator's world-frame inverse inertia against a principal-axis
  decomposition built by rotating vectors with quaternion products;
* the torque on a rotating sphere against Stokes' law 8 pi eta R^3 Omega,
  with R the hydrodynamic radius fitted from the Stokes drag of the same
  staircase sphere in a periodic array (Hasimoto 1959)."""
import copy
import math

import numpy as np
import pytest

import workloads as W
from oracle import OracleSim, coupling, rigid
from oracle.d3q19 import E, Q, W as WT


def _cross(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def _cell_centres(sim):
    nx, ny, nz = sim.dims
    c = np.arange(sim.N)
    return np.stack([c % nx + 0.5, (c // nx) % ny + 0.5, c // (nx * ny) + 0.5]).astype(float)


def _angular_momentum_terms(sim, df):
    # x x j over the fluid cells, j = sum_alpha e_alpha dF_alpha (the rest
    # weights carry no momentum); returns the per-cell terms of each component
    x = _cell_centres(sim)
    fluid = sim.flags == 0
    j = E.T.astype(float) @ df
    L = _cross(x, j)
    return [v[fluid] for v in L]


def _wall_torque_terms(sim):
    # momentum exchange with the halfway walls, about the origin: every
    # population f~ = w + dF~ that would leave through a wall comes back
    # reversed, handing 2 e_alpha f~_alpha to the wall at the fluid cell
    x = _cell_centres(sim)
    fluid = np.nonzero(sim.flags == 0)[0]
    out = [[], [], []]
    for a in range(1, Q):
        sel = fluid[sim.nbr[a, fluid] < 0]
        if sel.size == 0:
            continue
        s = 2.0 * (WT[a] + sim.dft[a, sel])
        f = [E[a, d] * s for d in range(3)]
        t = _cross([x[d][sel] for d in range(3)], f)
        for d in range(3):
            out[d].extend(t[d].tolist())
    return out


def test_per_step_angular_momentum_balance():
    # walls on every face, so that positions are unambiguous; two kinematic
    # bodies off the lattice points spin with prescribed Omega (V = 0, and
    # shapes that the rotation maps onto themselves, so no cell changes
    # side); random initial populations
    case = W.Case("spin", 22, 18, 16, 0.8, periodic=(False, False, False), bodies=[
        W.make_body(W.SPHERE, 3.1, 1.0, (6.3, 8.1, 7.7), kinematic=1, omega=(0.004, -0.003, 0.007)),
        # a tilted capsule spinning about its own axis (rotation about y by
        # 0.8 takes the body x axis to (cos 0.8, 0, -sin 0.8)): its cells stay
        W.make_body(W.CAPSULE, 2.2, 1.0, (15.4, 9.6, 8.3), h=1.7, kinematic=1,
                    omega=(0.006 * math.cos(0.8), 0.0, -0.006 * math.sin(0.8)),
                    quat=(math.cos(0.4), 0.0, math.sin(0.4), 0.0)),
    ])
    df0 = W.initial_populations(case, seed=5, amp=1e-4)
    sim = OracleSim(case, df0=df0)
    flags0 = sim.flags.copy()
    for _ in range(6):
        before = _angular_momentum_terms(sim, sim.df)
        sim.step()
        assert np.array_equal(sim.flags, flags0)
        after = _angular_momentum_terms(sim, sim.df)
        wall = _wall_torque_terms(sim)
        for d in range(3):
            body = []
            for b, bd in enumerate(sim.bodies):
                xf = _cross(bd["X"], sim.F[b])   # torque of F about the origin
                body += [sim.T[b][d], xf[d]]
            lhs = math.fsum(after[d].tolist() + (-before[d]).tolist())
            rhs = -math.fsum(body + wall[d])
            scale = math.fsum(np.abs(after[d]).tolist()) + math.fsum(np.abs(wall[d]).tolist())
            assert abs(lhs - rhs) < 1e-14 * scale, (d, lhs, rhs)
            # the torques are not trivially zero
            assert abs(rhs) > 1e-6 * scale
    # the bodies' own torque (about their centres) is nonzero and differs from
    # the torque about the origin, so a wrong lever-arm origin would show
    assert all(max(abs(v) for v in sim.T[b]) > 1e-6 for b in range(2))


@pytest.mark.parametrize("seed", range(4))
def test_geometric_torque_integer_form_equals_direct_sum(seed):
    # the part 2 w_alpha e_alpha of the link term and its torque, summed
    # directly over the links with float lever arms (cell centre minus body
    # position, minimum image on periodic axes), against the oracle's exact
    # integer form (S / 72 - f x G / 36)
    rng = np.random.default_rng(300 + seed)
    L = (30, 26, 24)
    periodic = (True, bool(seed % 2), False)
    shape = W.SPHERE if seed < 2 else W.CAPSULE
    # For a body with fluid all around, G and the geometric torque vanish
    # identically (the link set pairs up); a body cut by the z wall (cells
    # in its first layer) has links only on its fluid side, so both are
    # nonzero.  Near the periodic x face in half the cases, so that the
    # minimum image matters.
    pos = (float(rng.uniform(0.1, 2.0) if seed % 2 else rng.uniform(10, 20)), float(rng.uniform(10, 16)),
           float(rng.uniform(0.6, 2.4)))
    ang = float(rng.uniform(0, math.pi))
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    quat = (math.cos(ang / 2),) + tuple(float(v) * math.sin(ang / 2) for v in ax)
    body = W.make_body(shape, 3.3, 1.0, pos, h=2.1 if shape == W.CAPSULE else 0.0, quat=quat)
    case = W.Case("g", *L, 1.0, periodic=periodic, bodies=[body])
    sim = OracleSim(case)
    lc, ld, lb = sim.links
    y = sim.nbr[ld, lc]
    bd = sim.bodies[0]
    # rest state: dF~ = 0, rho = 1, body at rest -> F = G, T = geometric torque
    F, T = coupling.link_forces(ld, lb, y, np.zeros(len(ld)), np.ones(len(ld)), sim.bodies, sim.dims,
                                sim.periodic)
    nx, ny, nz = sim.dims
    cen = [y % nx + 0.5, (y // nx) % ny + 0.5, y // (nx * ny) + 0.5]
    r = []
    for d in range(3):
        v = cen[d] - bd["X"][d]
        if sim.periodic[d]:
            v = v - L[d] * np.round(v / L[d])
        r.append(v)
    g = [2.0 * WT[ld] * E[ld, d] for d in range(3)]
    G = [math.fsum(v.tolist()) for v in g]
    Td = [math.fsum(v.tolist()) for v in _cross(r, g)]
    assert max(abs(v) for v in G) > 0.05 and max(abs(v) for v in Td) > 0.05
    for d in range(3):
        assert abs(F[0][d] - G[d]) < 1e-14
        assert abs(T[0][d] - Td[d]) < 1e-13 * max(1.0, abs(Td[d]))


def _rotate(q, v):
    # q v q* with Hamilton products (independent of the rotation matrix)
    def mul(a, b):
        return [a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3],
                a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2],
                a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1],
                a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0]]
    qc = [q[0], -q[1], -q[2], -q[3]]
    return np.array(mul(mul(q, [0.0, *v]), qc)[1:])


def _free_capsule(quat):
    m, r, h = 400.0, 4.0, 4.0
    b = W.make_body(W.CAPSULE, r, m, (0.0, 0.0, 0.0), h=h, quat=quat)
    return {"shape": b.shape, "radius": r, "half_len": h, "mass": m, "inertia": list(b.inertia),
            "anchor": [0.0] * 3, "D": [0.0] * 3, "quat": list(quat), "V": [0.0] * 3, "Omega": [0.0] * 3,
            "kinematic": 0}


def test_one_step_under_torque_uses_the_world_frame_inertia():
    q = np.array([0.8, 0.3, -0.4, 0.33])
    q = q / np.linalg.norm(q)
    body = _free_capsule(q.tolist())
    Ip = body["inertia"]
    assert Ip[0] < Ip[1]   # the capsule is slimmer about its axis
    axes = [_rotate(q, e) for e in np.eye(3)]
    Iw = sum(Ip[p] * np.outer(axes[p], axes[p]) for p in range(3))
    T = np.array([0.3, -0.7, 0.45])
    F = [1e-3, -2e-3, 5e-4]
    rigid.integrate(body, F, T.tolist())
    want = np.linalg.solve(Iw, T)
    assert np.allclose(body["Omega"], want, rtol=1e-13, atol=0)
    # a transposed frame gives another answer: the test can tell them apart
    M = np.array(axes)          # row p is the world direction of principal axis p
    axes_t = [M[:, p] for p in range(3)]
    Iw_t = sum(Ip[p] * np.outer(axes_t[p], axes_t[p]) for p in range(3))
    assert np.abs(np.linalg.solve(Iw_t, T) - want).max() > 1e-3 * np.abs(want).max()
    assert np.allclose(body["V"], np.array(F) / 400.0, rtol=1e-15, atol=0)


@pytest.mark.parametrize("axis", [0, 1])
def test_constant_torque_about_a_principal_axis_spins_up_linearly(axis):
    # a torque along a principal axis of a rotated capsule keeps that axis
    # fixed while the body spins up, so Omega_n = n T / I_p exactly
    q = np.array([0.9, -0.2, 0.35, 0.1])
    q = q / np.linalg.norm(q)
    body = _free_capsule(q.tolist())
    a = _rotate(q, np.eye(3)[axis])
    T = (2e-2 * a).tolist()
    n = 60
    for _ in range(n):
        rigid.integrate(body, [0.0, 0.0, 0.0], T)
    want = n * np.array(T) / body["inertia"][axis]
    assert np.allclose(body["Omega"], want, rtol=1e-12, atol=1e-18)
    # the body has turned by a finite angle about that axis
    turned = _rotate(body["quat"], np.eye(3)[(axis + 1) % 3])
    assert np.abs(turned - _rotate(q, np.eye(3)[(axis + 1) % 3])).max() > 1e-3
    assert np.allclose(_rotate(body["quat"], np.eye(3)[axis]), a, atol=1e-12)


def _hydrodynamic_radius(L, r, tau, g, steps):
    # Stokes drag of the staircase sphere in a periodic cubic array
    # (Hasimoto 1959): F = 6 pi eta R U / K(phi); R fitted from the measured F
    body = W.make_body(W.SPHERE, r, 1.0, (L / 2.0, L / 2.0, L / 2.0), kinematic=True)
    case = W.Case("hasimoto", L, L, L, tau, periodic=(True, True, True), bodies=[body])
    sim = OracleSim(case, g=(g, 0.0, 0.0)).run(steps)
    f = sim.populations()
    u = (np.tensordot(E[:, 0], f, axes=(0, 0)) + 0.5 * g) / (1.0 + f.sum(0))
    fluid = (sim.flags == 0).reshape(L, L, L)
    U = u[fluid].sum() / L ** 3
    nu = (tau - 0.5) / 3.0
    target = sim.F[0][0] / (6.0 * math.pi * nu * U)

    def ratio(R):
        phi = 4.0 / 3.0 * math.pi * R ** 3 / L ** 3
        return R / (1.0 - 1.7601 * phi ** (1.0 / 3.0) + phi - 1.5593 * phi ** 2)

    lo, hi = 0.5 * r, 2.0 * r
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if ratio(mid) < target else (lo, mid)
    return 0.5 * (lo + hi)


@pytest.mark.slow
def test_rotating_sphere_torque_follows_stokes_law():
    # a kinematic sphere spinning at Omega about z in a periodic box: at
    # steady state the fluid resists with T = -8 pi eta R^3 Omega (Stokes),
    # eta = rho nu with rho = 1; the periodic images change this by about
    # the volume fraction (1% here).  The sign fixes the direction of
    # Omega x r in u_w and of the torque sum; the magnitude, within 3%, the
    # lever arm at which u_w and the torque are taken
    L, r, tau = 14, 2.0, 1.0
    Rh = _hydrodynamic_radius(L, r, tau, 1e-6, 3300)
    assert 0.85 * r < Rh < 1.1 * r
    Om = 1e-4
    for axis in (2, 0):
        omega = [0.0, 0.0, 0.0]
        omega[axis] = Om
        body = W.make_body(W.SPHERE, r, 1.0, (L / 2, L / 2, L / 2), kinematic=True, omega=tuple(omega))
        case = W.Case("spin", L, L, L, tau, periodic=(True, True, True), bodies=[body])
        sim = OracleSim(case).run(500)
        T = sim.T[0]
        stokes = -8.0 * math.pi * (tau - 0.5) / 3.0 * Rh ** 3 * Om
        assert math.isclose(T[axis], stokes, rel_tol=0.03), (T, stokes)
        assert all(abs(T[d]) < 1e-9 * abs(stokes) for d in range(3) if d != axis)
        assert max(abs(v) for v in sim.F[0]) < 1e-12 * abs(stokes)
