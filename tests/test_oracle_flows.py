"""Pins of the oracle against analytic flows: Couette flow driven by a moving
object (the moving bounce-back rule of Sec. 2.3), Poiseuille flow between
halfway bounce-back walls (Eq. lbm:bounce_back with the LBGK of Sec. 2.1), and
Stokes drag on a sphere in a periodic array (Hasimoto 1959), which pins the
momentum-exchange force of Eq. hydroF in magnitude."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import OracleSim
from oracle.d3q19 import E


def _velocity_x(sim, g=0.0):
    f = sim.populations()
    j = np.tensordot(E[:, 0], f, axes=(0, 0))
    rho = 1.0 + f.sum(0)
    return (j + 0.5 * g) / rho


@pytest.mark.parametrize("tau", [0.8, 1.0, 1.7])
def test_couette_profile_is_exactly_linear(tau):
    # fluid between a resting halfway wall at y = 0 and a kinematic slab whose
    # lower face is at y = H, moving at U along x: u(y) = U y / H for any tau
    U, H = 1e-3, 10
    c = 2 ** -0.5  # quaternion rotating local x onto +y
    slab = W.Body(shape=W.SLAB, radius=1.0, mass=1.0, anchor=(0.0, float(H), 0.0),
                  quat=(c, 0.0, 0.0, c), vel=(U, 0.0, 0.0), kinematic=True)
    case = W.Case("couette", 4, H + 2, 4, tau, periodic=(True, False, True), bodies=[slab])
    sim = OracleSim(case).run(3000)
    u = _velocity_x(sim)[0, :H, 0]
    y = np.arange(H) + 0.5
    assert np.max(np.abs(u - U * y / H)) < 1e-12 * U


@pytest.mark.parametrize("tau", [0.5 + math.sqrt(3) / 4, 1.0, 0.8])
def test_poiseuille_profile_with_halfway_slip(tau):
    # body-force driven channel flow between halfway bounce-back walls at
    # y = 0 and y = H: LBGK gives the parabola plus a tau-dependent slip,
    # u(y) = g/(2 nu) [y (H - y) + (16 L - 3)/12], L = (tau - 1/2)^2, nu = (tau - 1/2)/3,
    # exact to rounding; at tau = 1/2 + sqrt(3)/4 the slip vanishes
    g, H = 1e-6, 10
    case = W.Case("poiseuille", 4, H, 4, tau, periodic=(True, False, True))
    sim = OracleSim(case, g=(g, 0.0, 0.0)).run(3000)
    u = _velocity_x(sim, g)[0, :, 0]
    nu = (tau - 0.5) / 3.0
    lam = (tau - 0.5) ** 2
    y = np.arange(H) + 0.5
    exact = g / (2.0 * nu) * (y * (H - y) + (16.0 * lam - 3.0) / 12.0)
    assert np.max(np.abs(u - exact)) < 1e-12 * exact.max()
    # the wall friction balances the driving force exactly at steady state:
    # the momentum-exchange bookkeeping closes
    assert np.allclose(u, u[::-1], rtol=1e-13)


def _hasimoto_drag(L, r, tau, g, steps):
    body = W.make_body(W.SPHERE, r, 1.0, (L / 2.0, L / 2.0, L / 2.0), kinematic=True)
    case = W.Case("hasimoto", L, L, L, tau, periodic=(True, True, True), bodies=[body])
    sim = OracleSim(case, g=(g, 0.0, 0.0)).run(steps)
    u = _velocity_x(sim, g)
    fluid = (sim.flags == 0).reshape(L, L, L)
    U = u[fluid].sum() / L ** 3                # mean velocity of the suspension
    nu = (tau - 0.5) / 3.0
    F = sim.F[0][0]
    return F, U, nu, int(fluid.sum())


@pytest.mark.slow
def test_hasimoto_periodic_array_drag():
    # Stokes drag in a simple cubic array of spheres (Hasimoto 1959):
    #   F = 6 pi eta R U / K(phi), K = 1 - 1.7601 phi^(1/3) + phi - 1.5593 phi^2 + ...
    # The staircase sphere has an effective hydrodynamic radius R_h != r; fit it
    # on the largest box and predict the drag on the smaller ones.
    # tau = 1 keeps the viscosity-dependent offset of the bounce-back surface
    # small (at large tau it shrinks the effective radius well below r)
    tau, g, r = 1.0, 1e-6, 2.0
    # steps chosen so the start-up transient has decayed below 1e-4
    res = {L: _hasimoto_drag(L, r, tau, g, steps) for L, steps in ((10, 1200), (12, 1900), (14, 3300))}
    for L, (F, U, nu, nfl) in res.items():
        # steady state: the momentum-exchange force balances the body force
        assert math.isclose(F, g * nfl, rel_tol=1e-4)

    def K(phi):
        return 1.0 - 1.7601 * phi ** (1.0 / 3.0) + phi - 1.5593 * phi ** 2

    def drag_ratio(R, L):  # F / (6 pi eta U)
        phi = 4.0 / 3.0 * math.pi * R ** 3 / L ** 3
        return R / K(phi)

    F, U, nu, _ = res[14]
    target = F / (6.0 * math.pi * nu * U)
    lo, hi = 1.0, 4.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if drag_ratio(mid, 14) < target:
            lo = mid
        else:
            hi = mid
    Rh = 0.5 * (lo + hi)
    assert 0.8 * r < Rh < 1.25 * r
    for L in (10, 12):
        F, U, nu, _ = res[L]
        measured = F / (6.0 * math.pi * nu * U)
        assert math.isclose(measured, drag_ratio(Rh, L), rel_tol=0.03)


@pytest.mark.parametrize("every", [1, 7])
def test_time_average_of_steady_couette_flow(every):
    # the time average of a steady flow is the flow itself: the Couette
    # profile u = U y / H at every fluid cell, and no samples inside the slab
    U, H = 1e-3, 10
    c = 2 ** -0.5
    slab = W.Body(shape=W.SLAB, radius=1.0, mass=1.0, anchor=(0.0, float(H), 0.0),
                  quat=(c, 0.0, 0.0, c), vel=(U, 0.0, 0.0), kinematic=True)
    case = W.Case("couette", 4, H + 2, 4, 0.8, periodic=(True, False, True), bodies=[slab])
    sim = OracleSim(case).run(3000)
    start = sim.n
    sim.flow_average_begin(every).run(50)
    mean, count = sim.flow_average()
    samples = len([n for n in range(start, start + 50) if n % every == 0])
    y = np.arange(H) + 0.5
    assert np.max(np.abs(mean[0, :, :H, :] - (U * y / H)[None, :, None])) < 1e-12 * U
    assert np.max(np.abs(mean[1:])) < 1e-15 and not np.any(mean[:, :, H:, :])
    assert np.all(count[:, :H, :] == samples) and not np.any(count[:, H:, :])
