"""Rigid-body side of the coupled step (Sec. 2.2, Alg. 1; Sec. 3.1-3.3).

Readings of points the paper leaves open:

* Driving (Eqs. FB1-FB3).  Eq. FB3 prints sin(2 pi (t + phi)/T), but the
  cycling narrative of Sec. 3.3 and the protocol of Sec. 5.1 delay the right
  body's force by phi.  The oracle uses the delay:
      F_left  = -a sin(omega t),
      F_right =  a sin(omega t - psi),   psi = omega phi (the phase lag),
      F_mid   = -(F_left + F_right),
  all along the swimmer axis (x).  The paper's start-up protocol (right force
  held at zero until t = phi) is optional (``gate_lagged``); so are the
  switch-off steps of Sec. 5.1 (``off_left``, ``off_right``; the middle force
  stays the negative sum of the other two).
* Springs (Eqs. spring_i, damp_i, osci_i/j): with d = x_i - x_j and l = |d|,
  body i feels -k (l - l0) d/l - gamma (u_i - u_j) and body j the opposite.
  l0 is the centre-to-centre rest length; the damping acts on the full
  relative velocity.
* Time integration (Alg. 1, "update position and velocity") is not specified;
  the oracle uses semi-implicit (symplectic) Euler with dt = 1, one rigid-body
  step per lattice step, so the force of step n moves the body to step n+1
  (explicit coupling, Alg. 2):
      V += F_tot / m,  D += V,  Omega += I_w^-1 T_hydro,
      q  = normalize(q + 1/2 [0, Omega] (x) q),
  where D accumulates the displacement from the fixed anchor and I_w is the
  inertia tensor in world axes (gyroscopic term neglected).  Kinematic bodies
  keep their prescribed V and Omega; bodies with locked rotation
  (kinematic = 2) integrate V and D but keep their prescribed Omega (their
  torque is still computed).  The paper's swimmer bodies only move along the
  swimmer axis (Sec. 5.1); a capsule of the paper's equal-mass convention is
  lighter than the fluid it displaces, and for it the explicit rotational
  update of this integrator is unstable, so the capsule workloads lock it.  Bodies never touch, so the contact and
  constraint stages of Alg. 1 are empty (Sec. 3.1).
"""
from __future__ import annotations

import math

import numpy as np


def driving_forces(drive, n, nb, dtype=np.float64):
    """F_dri of Eqs. FB1-FB3 at step n (x components; module docstring)."""
    F = [[0.0, 0.0, 0.0] for _ in range(nb)]
    for dv in drive:
        a = dv["amplitude"]
        om = 2.0 * math.pi / dv["period"]
        psi = dv["phase_lag"]
        fl = -a * np.sin(om * n)
        fr = a * np.sin(om * n - psi)
        if dv["gate_lagged"] and om * n < np.real(psi):
            fr = 0.0 * fr
        if dv["off_left"] >= 0 and n >= dv["off_left"]:
            fl = 0.0 * fl
        if dv["off_right"] >= 0 and n >= dv["off_right"]:
            fr = 0.0 * fr
        fm = -(fl + fr)
        F[dv["left"]][0] = F[dv["left"]][0] + fl
        F[dv["right"]][0] = F[dv["right"]][0] + fr
        F[dv["middle"]][0] = F[dv["middle"]][0] + fm
    return F


def spring_forces(springs, bodies):
    """F_osci of Eqs. osci_i/j summed over all springs."""
    F = [[0.0, 0.0, 0.0] for _ in bodies]
    for s in springs:
        bi, bj = bodies[s["i"]], bodies[s["j"]]
        d = [(bi["anchor"][k] - bj["anchor"][k]) + (bi["D"][k] - bj["D"][k]) for k in range(3)]
        ell = np.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
        coef = -s["k"] * (ell - s["rest_len"]) / ell
        f = [coef * d[k] - s["gamma"] * (bi["V"][k] - bj["V"][k]) for k in range(3)]
        for k in range(3):
            F[s["i"]][k] = F[s["i"]][k] + f[k]
            F[s["j"]][k] = F[s["j"]][k] - f[k]
    return F


def rotation_matrix(q):
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def integrate(body, F_tot, T_hydro):
    """One semi-implicit Euler step of a body (Alg. 1, time integration)."""
    if body["kinematic"] != 1:
        m = body["mass"]
        body["V"] = [body["V"][k] + F_tot[k] / m for k in range(3)]
    if body["kinematic"] == 0:
        R = rotation_matrix(body["quat"])
        inv = np.diag([1.0 / v for v in body["inertia"]])
        Iw_inv = R @ inv @ R.T
        dO = Iw_inv @ np.array(T_hydro)
        body["Omega"] = [body["Omega"][k] + dO[k] for k in range(3)]
    body["D"] = [body["D"][k] + body["V"][k] for k in range(3)]
    O = body["Omega"]
    w, x, y, z = body["quat"]
    # [0, O] (x) q
    pw = -(O[0] * x + O[1] * y + O[2] * z)
    px = O[0] * w + (O[1] * z - O[2] * y)
    py = O[1] * w + (O[2] * x - O[0] * z)
    pz = O[2] * w + (O[0] * y - O[1] * x)
    q = [w + 0.5 * pw, x + 0.5 * px, y + 0.5 * py, z + 0.5 * pz]
    nrm = np.sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3])
    body["quat"] = [v / nrm for v in q]
    body["X"] = [body["anchor"][k] + body["D"][k] for k in range(3)]
