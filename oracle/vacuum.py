"""The swimmer in vacuum (Sec. 4): the rigid-body side of Alg. 2 with no
fluid, and the closed-form solution of the resulting linear recurrence.

``run`` advances the bodies step by step with the oracle's own driving
(Eqs. FB1-FB3), spring-damper forces (Eqs. osci_i/j) and integrator (Alg. 1,
unit time step), the hydrodynamic force and torque being zero.

For one three-body swimmer along x (bodies ordered middle, left, right;
springs joining the middle body to each outer one) the step is linear in the
state s = (D, V) of the x displacements and velocities:
    V' = V + (K D + G V + F(n)) / m,   D' = D + V',
i.e. s_{n+1} = M s_n + c(n).  With sinusoidal driving c(n) = Re(c e^{i w n})
the solution from rest is
    s_n = Re(s_hat e^{i w n}) - M^n Re(s_hat),   s_hat = (e^{i w} I - M)^{-1} c,
which ``exact`` evaluates (M^n by repeated squaring: M has a Jordan block at
1, the free translation).  Its steady amplitude |s_hat| traces the resonance
curve of Fig. vacuumVal2.
"""
from __future__ import annotations

import numpy as np

from . import rigid
from .sim import _body_state


def run(case, steps, record=None):
    """Advance ``case``'s bodies ``steps`` steps in vacuum.  Returns the x
    displacement and velocity of every body after every step, with shape
    (steps, bodies, 2); ``record`` (a set of step indices) keeps only those."""
    bodies = [_body_state(b, float) for b in case.bodies]
    for b in bodies:
        b["X"] = [b["anchor"][k] + b["D"][k] for k in range(3)]
    springs = [dict(i=s.i, j=s.j, k=s.k, gamma=s.gamma, rest_len=s.rest_len) for s in case.springs]
    drives = [dict(left=d.left, middle=d.middle, right=d.right, amplitude=d.amplitude,
                   period=d.period, phase_lag=d.phase_lag, gate_lagged=d.gate_lagged,
                   off_left=d.off_left, off_right=d.off_right) for d in case.drives]
    hist = []
    for n in range(steps):
        Fd = rigid.driving_forces(drives, n, len(bodies))
        Fs = rigid.spring_forces(springs, bodies)
        for b, body in enumerate(bodies):
            Ft = [(0.0 + Fd[b][k]) + Fs[b][k] for k in range(3)]
            rigid.integrate(body, Ft, [0.0, 0.0, 0.0])
        if record is None or n in record:
            hist.append([[body["D"][0], body["V"][0]] for body in bodies])
    return np.array(hist)


def linear_system(m, k, g):
    """The step matrix M of the three-body chain (module docstring)."""
    K = np.array([[-2 * k, k, k], [k, -k, 0.0], [k, 0.0, -k]])
    G = np.array([[-2 * g, g, g], [g, -g, 0.0], [g, 0.0, -g]])
    I = np.eye(3)
    return np.block([[I + K / m, I + G / m], [K / m, I + G / m]])


def steady_response(m, k, g, a, w, psi):
    """Complex amplitude s_hat of the steady state under the ungated driving
    -a sin(w n) (left), a sin(w n - psi) (right), minus their sum (middle)."""
    M = linear_system(m, k, g)
    Fl = 1j * a                       # -a sin(wn) = Re(i a e^{iwn})
    Fr = -1j * a * np.exp(-1j * psi)  # a sin(wn - psi) = Re(-i a e^{-i psi} e^{iwn})
    Fc = np.array([-(Fl + Fr), Fl, Fr]) / m
    return np.linalg.solve(np.exp(1j * w) * np.eye(6) - M, np.concatenate([Fc, Fc]))


def exact(m, k, g, a, w, psi, n):
    """State (D of middle, left, right; V likewise) after step n - 1, i.e. s_n,
    of the swimmer started at rest under the ungated driving."""
    M = linear_system(m, k, g)
    s_hat = steady_response(m, k, g, a, w, psi)
    return np.real(s_hat * np.exp(1j * w * n)) - np.linalg.matrix_power(M, n) @ np.real(s_hat)
