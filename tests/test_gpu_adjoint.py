"""Hand-written adjoint of the coupled step (lbm_adjoint) against the CPU
oracle's complex-step tangent and against central finite differences of the
GPU forward run."""
import copy
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import OracleSim

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PARAMS = ("amplitude", "phase_lag", "k")


def _tiny():
    b, s, d = W.swimmer((12.0, 8.0, 8.0), r=2.0, l0=(7.0, 7.0), k=0.05, gamma=0.01,
                        amplitude=5e-3, period=20.0, phase_lag=1.1)
    return W.Case("tiny", 24, 16, 16, 0.9, bodies=b, springs=s, drives=[d], steps=30)


def _with(case, **kw):
    c = copy.deepcopy(case)
    for d in c.drives:
        if "amplitude" in kw:
            d.amplitude = kw["amplitude"]
        if "phase_lag" in kw:
            d.phase_lag = kw["phase_lag"]
    for s in c.springs:
        if "k" in kw:
            s.k = kw["k"]
    return c


def _gpu_J(case, storage):
    from paper_1108_0786_amd.sim import Sim
    sim = Sim(case, storage=storage)
    sim.step(case.steps)
    J = sim.centroid_displacement()
    sim.close()
    return J


@pytest.mark.parametrize("average", [False, True])
def test_adjoint_matches_oracle_complex_step_tiny(average):
    # plain explicit coupling and the two-step force mean
    from paper_1108_0786_amd.sim import Sim
    case = _tiny()
    case.force_average = average
    base = {"amplitude": 5e-3, "phase_lag": 1.1, "k": 0.05}
    print(f"[gpu] adjoint tiny {case.name} {case.steps} steps, force mean {average}", flush=True)
    sim = Sim(case, storage="f64")
    J, grad = sim.adjoint(case.steps, checkpoint_every=7)
    sim.close()
    J_orc = OracleSim(case).run(case.steps).centroid_displacement()
    want = []
    for i, p in enumerate(PARAMS):
        h = 1e-20 * base[p]
        orc = OracleSim(case, dtype=np.complex128, params={p: base[p] + 1j * h}).run(case.steps)
        want.append(orc.centroid_displacement().imag / h)
    want = np.array(want)
    print(f"[gpu] J {J:.6e} (oracle {J_orc:.6e}); grad {grad} vs {want}", flush=True)
    assert math.isclose(J, J_orc, rel_tol=1e-12)
    assert np.allclose(grad, want, rtol=1e-8, atol=0)


def test_adjoint_leaves_the_forward_state():
    # after lbm_adjoint the context is where lbm_step(nsteps) would leave it
    from paper_1108_0786_amd.sim import Sim
    case = _tiny()
    a = Sim(case, storage="f32", traj_cap=4)
    a.adjoint(case.steps, checkpoint_every=8)
    b = Sim(case, storage="f32", traj_cap=4)
    b.step(case.steps)
    assert np.array_equal(a.populations(), b.populations())
    assert a.bodies() == b.bodies()
    a.step(5)
    b.step(5)
    assert np.array_equal(a.populations(), b.populations())


def test_adjoint_case_against_finite_differences_and_tangent():
    # 128x64x64, two periods of 500 steps, FP32 populations, checkpoints every 50 steps
    from paper_1108_0786_amd.autograd import swimmer_displacement
    case = W.adjoint_case(storage="f32")
    base = {"amplitude": case.drives[0].amplitude, "phase_lag": case.drives[0].phase_lag,
            "k": case.springs[0].k}
    print(f"[gpu] adjoint {case.name} {case.steps} steps", flush=True)
    theta = torch.tensor([base[p] for p in PARAMS], dtype=torch.float64, requires_grad=True)
    J = swimmer_displacement(theta, case, case.steps, storage="f32", checkpoint_every=50)
    J.backward()
    grad = theta.grad.numpy()
    # central differences of the FP64 GPU forward run, h = 1e-3 relative
    fd = []
    for p in PARAMS:
        h = 1e-3 * base[p]
        jp = _gpu_J(_with(case, **{p: base[p] + h}), "f64")
        jm = _gpu_J(_with(case, **{p: base[p] - h}), "f64")
        fd.append((jp - jm) / (2 * h))
    fd = np.array(fd)
    print(f"[gpu] J {J.item():.6e}; adjoint {grad}; central differences {fd}", flush=True)
    scale = np.abs(fd)
    assert np.all(np.abs(grad - fd) <= 1e-4 * scale + 1e-12 * np.abs(fd).max())
    # the oracle's complex-step tangent, computed once by tests/golden/make_goldens.py
    files = [os.path.join(GOLD, f"adjoint_tangent_{p}.json") for p in PARAMS]
    if all(os.path.exists(f) for f in files):
        tan = np.array([json.load(open(f))["dJ"] for f in files])
        print(f"[gpu] oracle tangent {tan}", flush=True)
        assert np.all(np.abs(grad - tan) <= 1e-4 * np.abs(tan))
