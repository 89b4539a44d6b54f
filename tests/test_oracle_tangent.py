"""The oracle's complex-step tangent (complex128 run with an imaginary
perturbation of one parameter) agrees with central finite differences of the
real oracle; both differentiate the swimmer's net displacement."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import OracleSim


def _tiny_swimmer():
    b, s, d = W.swimmer((12.0, 8.0, 8.0), r=2.0, l0=(7.0, 7.0), k=0.05, gamma=0.01,
                        amplitude=5e-3, period=20.0, phase_lag=1.1)
    return W.Case("tiny", 24, 16, 16, 0.9, bodies=b, springs=s, drives=[d], steps=30)


def _J(case, params, dtype=np.float64):
    sim = OracleSim(case, dtype=dtype, params=params)
    sim.run(case.steps)
    return sim.centroid_displacement()


@pytest.mark.parametrize("name,base", [("amplitude", 5e-3), ("phase_lag", 1.1), ("k", 0.05)])
def test_complex_step_matches_central_difference(name, base):
    case = _tiny_swimmer()
    h = 1e-20 * base
    J_cs = _J(case, {name: base + 1j * h}, np.complex128)
    dJ_cs = J_cs.imag / h
    # central difference with a relative step of 1e-3 (error O(h^2))
    hf = 1e-3 * base
    dJ_fd = (_J(case, {name: base + hf}) - _J(case, {name: base - hf})) / (2 * hf)
    assert abs(dJ_cs) > 0
    assert math.isclose(dJ_cs, dJ_fd, rel_tol=1e-4)
    # the real part of the complex run is the real run
    assert math.isclose(J_cs.real, _J(case, {name: base}), rel_tol=1e-13)
