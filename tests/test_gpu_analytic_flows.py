"""Analytic flows through the C-ABI (the same checks that pin the oracle,
now on the GPU path): Couette flow driven by a moving kinematic slab (the
moving bounce-back of Sec. 2.3), Poiseuille flow driven by the test-only
uniform body force between halfway bounce-back walls (Eq. lbm:bounce_back),
and the Stokes drag of a sphere in a periodic array (Eq. hydroF, Hasimoto
1959), each in FP64 with two buffers and in place.

Asserted: the Couette profile is linear and the Poiseuille profile is the
LBGK parabola with its tau-dependent slip, both to 1e-12 of their scale; the
sphere array's momentum-exchange force balances the body force on the fluid
at steady state, and force, mean velocity and populations equal the
oracle's to 1e-12."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import OracleSim
from oracle.d3q19 import E

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _sim(case, **kw):
    from paper_1108_0786_amd.sim import Sim
    return Sim(case, device="cuda:0", storage="f64", **kw)


def _velocity_x(f, g=0.0):
    j = np.tensordot(E[:, 0], f, axes=(0, 0))
    rho = 1.0 + f.sum(0)
    return (j + 0.5 * g) / rho


@pytest.mark.parametrize("streaming", [0, 1])
@pytest.mark.parametrize("tau", [0.8, 1.0, 1.7])
def test_couette_profile_is_exactly_linear(tau, streaming):
    U, H = 1e-3, 10
    c = 2 ** -0.5  # quaternion rotating local x onto +y
    slab = W.Body(shape=W.SLAB, radius=1.0, mass=1.0, anchor=(0.0, float(H), 0.0),
                  quat=(c, 0.0, 0.0, c), vel=(U, 0.0, 0.0), kinematic=True)
    case = W.Case("couette", 4, H + 2, 4, tau, periodic=(True, False, True), bodies=[slab])
    print(f"[gpu] Couette, tau {tau}, streaming {streaming}", flush=True)
    sim = _sim(case, tune={"streaming": streaming})
    sim.step(3001)
    sim.status()
    u = _velocity_x(sim.populations())[:, :H, :]
    y = np.arange(H) + 0.5
    assert np.max(np.abs(u - (U * y / H)[None, :, None])) < 1e-12 * U
    sim.close()


@pytest.mark.parametrize("streaming", [0, 1])
@pytest.mark.parametrize("tau", [0.5 + math.sqrt(3) / 4, 1.0, 0.8])
def test_poiseuille_profile_with_halfway_slip(tau, streaming):
    g, H = 1e-6, 10
    case = W.Case("poiseuille", 4, H, 4, tau, periodic=(True, False, True))
    print(f"[gpu] Poiseuille, tau {tau:.4f}, streaming {streaming}", flush=True)
    sim = _sim(case, tune={"streaming": streaming}, body_force=(g, 0.0, 0.0))
    sim.step(3001)
    u = _velocity_x(sim.populations(), g)[0, :, 0]
    nu = (tau - 0.5) / 3.0
    lam = (tau - 0.5) ** 2
    y = np.arange(H) + 0.5
    exact = g / (2.0 * nu) * (y * (H - y) + (16.0 * lam - 3.0) / 12.0)
    assert np.max(np.abs(u - exact)) < 1e-12 * exact.max()
    assert np.allclose(u, u[::-1], rtol=1e-13)
    sim.close()


@pytest.mark.parametrize("streaming", [0, 1])
def test_sphere_array_drag_against_oracle(streaming):
    L, r, tau, g, steps = 10, 2.0, 1.0, 1e-6, 1201
    body = W.make_body(W.SPHERE, r, 1.0, (L / 2.0, L / 2.0, L / 2.0), kinematic=True)
    case = W.Case("hasimoto", L, L, L, tau, periodic=(True, True, True), bodies=[body])
    print(f"[gpu] sphere array, streaming {streaming}", flush=True)
    orc = OracleSim(case, g=(g, 0.0, 0.0)).run(steps)
    sim = _sim(case, traj_cap=steps, tune={"streaming": streaming}, body_force=(g, 0.0, 0.0))
    sim.step(steps)
    F = sim.trajectory()[steps - 1, 0, 9]
    Fo = orc.F[0][0]
    assert abs(F - Fo) < 1e-12 * abs(Fo)
    orc.map_next()
    pg, po = sim.populations(), orc.populations()
    assert np.abs(pg - po).max() < 1e-12 * np.abs(po).max()
    fluid = (orc.flags == 0).reshape(L, L, L)
    U = _velocity_x(pg, g)[fluid].sum() / L ** 3
    Uo = _velocity_x(po, g)[fluid].sum() / L ** 3
    assert abs(U - Uo) < 1e-12 * abs(Uo)
    # steady state: the momentum exchange balances the force on the fluid
    assert math.isclose(F, g * int(fluid.sum()), rel_tol=1e-4)
    sim.close()


def test_force_refuses_flow_average():
    from paper_1108_0786_amd import _abi
    case = W.Case("poiseuille", 4, 10, 4, 1.0, periodic=(True, False, True))
    sim = _sim(case, body_force=(1e-6, 0.0, 0.0))
    with pytest.raises(_abi.LbmError) as e:
        sim.flow_average_begin(1)
    assert e.value.code == _abi.LBM_E_STATE
    sim.close()
