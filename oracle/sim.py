"""The coupled LBM / rigid-body step for swimmers, Alg. 2 of Sec. 2.3.

One step n, in the order of Alg. 2:

 1. map every body onto the lattice (flag field), with the flag changes of
    Sec. 2.3 (refill of uncovered cells, covered cells dropped), and collect
    the boundary links;
 2. collide and stream every fluid cell (Sec. 2.1), with halfway bounce-back
    at the channel walls and moving bounce-back at object cells;
 3. sum the momentum-exchange force and torque of every object (Eq. hydroF);
 4. add the driving forces (Eqs. FB1-FB3);
 5. rigid-body step (Alg. 1): spring-damper forces (Eqs. osci_i/j), total
    force (Eqs. totalF, totalFSwimmer), time integration.

Force averaging (a reading; the paper is silent on it).  With
``case.force_average`` the rigid-body step of step n uses the mean of the
hydrodynamic force and torque of steps n and n-1 (those of step -1 are
zero).  For tau < 1 the over-relaxed collision makes the fluid's response to
a body velocity that alternates from step to step add up coherently, and for
light enough bodies the explicit coupling then amplifies that period-2 mode;
the two-step mean removes it exactly.  The recorded F and T stay the
momentum-exchange sums of the step itself.

Time-averaged flow field (Sec. 6, Fig. flowfields13: flow fields averaged
over five swimming cycles).  A reading, as the paper gives only the figure:
the average at a cell is the mean of the fluid velocity u = j / rho of
Sec. 2.1 over the sampled steps in which the cell is fluid.  A step n is
sampled when n % every == 0; its velocity is that of the pre-collision state
of step n after its mapping, the state step 2 starts from.

The state is held in deviation form (oracle.lbm).  With ``dtype=complex128``
the same code runs the complex-step tangent: a parameter given an imaginary
perturbation i h propagates so that Im(J)/h is dJ/dparameter to rounding
(Squire and Trapp 1998); flags use real parts only.
"""
from __future__ import annotations

import copy
import math

import numpy as np

from . import coupling, lbm, rigid


def _body_state(b, dtype):
    return {
        "shape": int(b.shape), "radius": float(b.radius), "half_len": float(b.half_len),
        "mass": float(b.mass), "inertia": [float(v) for v in b.inertia],
        "anchor": [float(v) for v in b.anchor],
        "D": [dtype(v) for v in b.disp], "quat": [dtype(v) for v in b.quat],
        "V": [dtype(v) for v in b.vel], "Omega": [dtype(v) for v in b.omega],
        "kinematic": int(b.kinematic),
    }


class OracleSim:
    """Alg. 2 on one box.  ``case`` is a ``workloads.Case``."""

    def __init__(self, case, dtype=np.float64, df0=None, g=None, params=None):
        self.case = case
        self.dtype = dtype
        self.dims = (case.nx, case.ny, case.nz)
        self.periodic = tuple(bool(p) for p in case.periodic)
        self.N = case.nx * case.ny * case.nz
        self.tau = case.tau
        self.g = g
        self.nbr = lbm.neighbour_table(case.nx, case.ny, case.nz, self.periodic)
        self.bodies = [_body_state(b, dtype) for b in case.bodies]
        for body in self.bodies:
            body["X"] = [body["anchor"][k] + body["D"][k] for k in range(3)]
        self.springs = [dict(i=s.i, j=s.j, k=s.k, gamma=s.gamma, rest_len=s.rest_len)
                        for s in case.springs]
        self.drives = [dict(left=d.left, middle=d.middle, right=d.right, amplitude=d.amplitude,
                            period=d.period, phase_lag=d.phase_lag, gate_lagged=d.gate_lagged,
                            off_left=d.off_left, off_right=d.off_right) for d in case.drives]
        if params:
            # complex-step / finite-difference overrides: amplitude, phase_lag, k
            for d in self.drives:
                for key in ("amplitude", "phase_lag"):
                    if key in params:
                        d[key] = params[key]
            for s in self.springs:
                if "k" in params:
                    s["k"] = params["k"]
        self.df = np.zeros((19, self.N), dtype=dtype)
        if df0 is not None:
            self.df[:] = np.asarray(df0).reshape(19, self.N)
        # Before the first map every cell is fluid; the first map only covers.
        self.flags = np.zeros(self.N, dtype=np.uint8)
        self.n = 0
        self.traj = []
        self.force_average = bool(getattr(case, "force_average", False))
        self.F_prev = [[0.0, 0.0, 0.0] for _ in self.bodies]
        self.T_prev = [[0.0, 0.0, 0.0] for _ in self.bodies]
        self.flow_every = 0
        self.remap()

    # -- step 1 ------------------------------------------------------------
    def remap(self):
        new = coupling.map_bodies(self.bodies, self.dims, self.periodic)
        self.last_changes = coupling.refill(self.df, self.flags, new, self.nbr, self.bodies,
                                            self.dims, self.periodic)
        self.flags = new
        self.links = coupling.links(new, self.nbr)

    def map_next(self):
        """Apply the mapping of the next step now (step 1 of Alg. 2 for step n,
        which the next call of ``step`` would do first and then find nothing to
        change).  State compared at a step boundary is taken after it."""
        self.remap()
        return self

    def wall_velocity(self, b, cells):
        return coupling.wall_velocity(self.bodies[b], cells, self.dims, self.periodic)

    # -- one step of Alg. 2 -----------------------------------------------------
    def step(self):
        self.remap()
        dft, rho, u = lbm.collide(self.df, self.tau, self.g)
        self.dft, self.rho = dft, rho
        if self.flow_every and self.n % self.flow_every == 0:
            fluid = self.flags == 0
            for d in range(3):
                self.flow_sum[d][fluid] = self.flow_sum[d][fluid] + u[d][fluid]
            self.flow_count[fluid] += 1
        new = lbm.stream_bounce_back(dft, rho, self.flags, self.nbr, self.wall_velocity)
        lc, ld, lb = self.links
        F, T = coupling.momentum_exchange(lc, ld, lb, dft, rho, self.bodies, self.dims,
                                          self.periodic, self.nbr)
        nb = len(self.bodies)
        Fd = rigid.driving_forces(self.drives, self.n, nb)
        Fs = rigid.spring_forces(self.springs, self.bodies)
        for b, body in enumerate(self.bodies):
            if self.force_average:
                Fh = [0.5 * (F[b][k] + self.F_prev[b][k]) for k in range(3)]
                Th = [0.5 * (T[b][k] + self.T_prev[b][k]) for k in range(3)]
            else:
                Fh, Th = F[b], T[b]
            Ft = [(Fh[k] + Fd[b][k]) + Fs[b][k] for k in range(3)]
            rigid.integrate(body, Ft, Th)
        self.F_prev = [list(v) for v in F]
        self.T_prev = [list(v) for v in T]
        self.df = new
        self.F, self.T = F, T
        self.traj.append({
            "n": self.n, "F": [list(v) for v in F], "T": [list(v) for v in T],
            "D": [list(b["D"]) for b in self.bodies], "V": [list(b["V"]) for b in self.bodies],
            "Omega": [list(b["Omega"]) for b in self.bodies],
            "quat": [list(b["quat"]) for b in self.bodies],
        })
        self.n += 1

    def run(self, steps):
        for _ in range(steps):
            self.step()
        return self

    # -- observables ---------------------------------------------------------
    def populations(self):
        """Deviations dF with shape (19, nz, ny, nx); zero inside objects."""
        return self.df.reshape(19, self.dims[2], self.dims[1], self.dims[0])

    def flow_average_begin(self, every):
        """Clear the sums of the time-averaged flow and sample every
        ``every``-th step from now on (module docstring); 0 stops sampling."""
        self.flow_every = int(every)
        if every:
            self.flow_sum = np.zeros((3, self.N), dtype=self.dtype)
            self.flow_count = np.zeros(self.N, dtype=np.int64)
        return self

    def flow_average(self):
        """(mean fluid velocity with shape (3, nz, ny, nx), zero where a cell
        was never fluid in a sample; sample counts with shape (nz, ny, nx))."""
        shape = (self.dims[2], self.dims[1], self.dims[0])
        mean = np.zeros((3, self.N), dtype=self.dtype)
        seen = self.flow_count > 0
        for d in range(3):
            mean[d][seen] = self.flow_sum[d][seen] / self.flow_count[seen]
        return mean.reshape((3,) + shape), self.flow_count.reshape(shape)

    def centroid_displacement(self):
        """Mean x displacement of the bodies (equal masses): the swimmer's
        net displacement since t = 0."""
        return sum(b["D"][0] for b in self.bodies) / len(self.bodies)


def run_case(case, steps=None, **kw):
    sim = OracleSim(case, **kw)
    sim.run(case.steps if steps is None else steps)
    return sim
