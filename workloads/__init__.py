"""Seeded synthetic workloads for the three-bead swimmer step.

This module only *describes* inputs: box shapes, relaxation times, body
geometry and placement, spring and driving parameters, and the seeded random
draws of the parameter sweeps.  It holds none of the method's arithmetic, so
both the CPU oracle and the GPU binding can take their inputs from here without
sharing any code of the method itself.

Conventions (the paper states none of them in code form):

* D3Q19 lattice, cells ``(i, j, k)`` with ``i`` fastest, linear index
  ``i + nx*(j + ny*k)``, cell centre ``(i+0.5, j+0.5, k+0.5)``.
* The swimmer axis is x.  Body order follows the paper's naming of the
  three-sphere device (Sec. 3.1): index 0 is the middle body B1, index 1 the
  left body B2 (at -x), index 2 the right body B3 (at +x).
* Spring rest lengths are centre-to-centre distances (Eq. spring_i).
* Bead mass follows the paper's design study (Sec. 5.1): 5.44e-13 kg for a
  4 um sphere in a fluid of density 1360 kg/m^3 gives m = 400 lattice units at
  r = 4; other radii scale as m = 400 (r/4)^3, and every body of one swimmer
  gets the same mass (capsules included, as in Sec. 5.1).
"""
from __future__ import annotations

import dataclasses
import json
import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

SPHERE, CAPSULE, SLAB = 0, 1, 2
STORAGE = {"f64": 0, "f32": 1, "f16s": 2, "bf16s": 3}


@dataclass
class Body:
    shape: int = SPHERE
    radius: float = 3.0
    half_len: float = 0.0          # capsule: half the cylinder length
    mass: float = 1.0
    inertia: Tuple[float, float, float] = (1.0, 1.0, 1.0)  # body frame, axis = local x
    anchor: Tuple[float, float, float] = (0.0, 0.0, 0.0)   # fixed reference position
    disp: Tuple[float, float, float] = (0.0, 0.0, 0.0)     # displacement from anchor
    quat: Tuple[float, float, float, float] = (1.0, 0.0, 0.0, 0.0)  # (w, x, y, z)
    vel: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    omega: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    kinematic: int = 0             # 0 free; 1 prescribed V and Omega; 2 prescribed Omega (rotation locked)


@dataclass
class Spring:
    i: int
    j: int
    k: float
    gamma: float
    rest_len: float                # centre-to-centre


@dataclass
class Drive:
    left: int
    middle: int
    right: int
    amplitude: float
    period: float
    phase_lag: float               # radians; the right body's force lags by this
    gate_lagged: bool = False      # right-body force held at 0 until omega*t >= phase_lag
    off_left: int = -1             # step from which the left force is switched off (-1: never)
    off_right: int = -1            # step from which the right force is switched off


@dataclass
class Case:
    name: str
    nx: int
    ny: int
    nz: int
    tau: float
    periodic: Tuple[bool, bool, bool] = (True, False, False)
    bodies: List[Body] = field(default_factory=list)
    springs: List[Spring] = field(default_factory=list)
    drives: List[Drive] = field(default_factory=list)
    steps: int = 0
    storage: str = "f64"
    shift_log2: int = 16          # scale exponent of the 16-bit storage formats
    force_average: bool = False   # bodies move with the mean of the last two hydrodynamic sums
    note: str = ""

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    def to_json(self) -> str:
        return json.dumps(dataclasses.asdict(self), sort_keys=True)


def bead_mass(r: float) -> float:
    """Bead mass in lattice units, m = 400 (r/4)^3 (design-study density)."""
    return 400.0 * (r / 4.0) ** 3


def sphere_inertia(m: float, r: float) -> Tuple[float, float, float]:
    i = 0.4 * m * r * r
    return (i, i, i)


def capsule_inertia(m: float, r: float, h: float) -> Tuple[float, float, float]:
    """Uniform solid capsule (cylinder of length 2h plus two hemispherical caps)
    of total mass m; returns (axial, transverse, transverse)."""
    vc = math.pi * r * r * 2.0 * h
    vs = 4.0 / 3.0 * math.pi * r ** 3
    mc = m * vc / (vc + vs)
    ms = m * vs / (vc + vs)
    H = 2.0 * h
    ia = mc * r * r / 2.0 + ms * 2.0 * r * r / 5.0
    it = mc * (H * H / 12.0 + r * r / 4.0) + ms * (2.0 * r * r / 5.0 + H * H / 4.0 + 3.0 * H * r / 8.0)
    return (ia, it, it)


def make_body(shape: int, r: float, m: float, pos, h: float = 0.0, **kw) -> Body:
    inertia = sphere_inertia(m, r) if shape == SPHERE else capsule_inertia(m, r, h)
    return Body(shape=shape, radius=float(r), half_len=float(h), mass=float(m),
                inertia=inertia, anchor=tuple(float(v) for v in pos), **kw)


def swimmer(centre, shapes=(SPHERE, SPHERE, SPHERE), r: float = 3.0, h: float = 0.0,
            l0: Tuple[float, float] = (10.0, 10.0), k: float = 0.05, gamma: float = 0.01,
            mass: Optional[float] = None, amplitude: float = 2e-4, period: float = 200.0,
            phase_lag: float = math.pi / 2, base: int = 0, **drive_kw):
    """Three bodies on the x axis, middle body at ``centre``.

    ``shapes`` lists (middle, left, right); ``l0`` = (left arm, right arm)
    centre-to-centre rest lengths.  Returns (bodies, springs, drive); body
    indices are offset by ``base`` so several swimmers can share one box."""
    m = bead_mass(r) if mass is None else mass
    cx, cy, cz = centre
    hm, hl, hr = [(h if s == CAPSULE else 0.0) for s in shapes]
    bodies = [
        make_body(shapes[0], r, m, (cx, cy, cz), hm),
        make_body(shapes[1], r, m, (cx - l0[0], cy, cz), hl),
        make_body(shapes[2], r, m, (cx + l0[1], cy, cz), hr),
    ]
    springs = [Spring(base + 1, base + 0, k, gamma, l0[0]),
               Spring(base + 2, base + 0, k, gamma, l0[1])]
    drive = Drive(left=base + 1, middle=base + 0, right=base + 2, amplitude=amplitude,
                  period=period, phase_lag=phase_lag, **drive_kw)
    return bodies, springs, drive


# --------------------------------------------------------------------------
# The five benchmark workloads
# --------------------------------------------------------------------------

def plain_f64_small() -> Case:
    """48x32x32, tau 1, r=3 three-sphere swimmer, 400 steps, FP64 (seed 0, nothing drawn)."""
    b, s, d = swimmer((24.0, 16.0, 16.0), r=3.0, l0=(10.0, 10.0), k=0.05, gamma=0.01,
                      amplitude=2e-4, period=200.0, phase_lag=math.pi / 2)
    return Case("plain_f64_48x32x32", 48, 32, 32, 1.0, bodies=b, springs=s, drives=[d],
                steps=400, storage="f64")


def plain_at_scale(storage: str = "f32", seed: int = 0, periods: int = 20) -> Case:
    """256x128x128, tau 0.8, r=6 swimmer, rest length 24, amplitude ~ U[1e-4,5e-4]."""
    rng = np.random.default_rng(seed)
    a = float(rng.uniform(1e-4, 5e-4))
    b, s, d = swimmer((128.0, 64.0, 64.0), r=6.0, l0=(24.0, 24.0), k=0.05, gamma=0.01,
                      amplitude=a, period=1000.0, phase_lag=math.pi / 2)
    return Case("plain_256x128x128", 256, 128, 128, 0.8, bodies=b, springs=s, drives=[d],
                steps=periods * 1000, storage=storage)


def capsule_swimmer(nx: int, ny: int, nz: int, design: str = "SCS", storage: str = "f32",
                    steps: int = 5000, shift_log2: int = 16) -> Case:
    """Capsule variant: r=5 bodies, capsules with cylinder length 10 parallel to x,
    surface gap 10 between neighbours; ``design`` is 'SCS' or 'CCC' (middle is
    the second letter).  Every body keeps the sphere's mass (Sec. 5.1), so a
    capsule is lighter than the fluid it displaces; the bodies' rotation is
    locked (they move along the swimmer axis only, as in Sec. 5.1), and they
    move with the two-step mean of the hydrodynamic force, without which the
    light capsules' translation is unstable at tau = 0.7."""
    r, h, gap = 5.0, 5.0, 10.0
    kinds = {"S": SPHERE, "C": CAPSULE}
    left, mid, right = (kinds[c] for c in design)
    ext = {SPHERE: r, CAPSULE: r + h}
    l_left = ext[left] + ext[mid] + gap
    l_right = ext[right] + ext[mid] + gap
    b, s, d = swimmer((nx / 2.0, ny / 2.0, nz / 2.0), shapes=(mid, left, right), r=r, h=h,
                      l0=(l_left, l_right), k=0.05, gamma=0.01, mass=bead_mass(r),
                      amplitude=3e-4, period=1000.0, phase_lag=math.pi / 2)
    for body in b:
        body.kinematic = 2
    return Case(f"capsule_{design}_{nx}x{ny}x{nz}", nx, ny, nz, 0.7, bodies=b, springs=s,
                drives=[d], steps=steps, storage=storage, shift_log2=shift_log2, force_average=True)


def capsule_full(design: str = "SCS", storage: str = "f32") -> Case:
    return capsule_swimmer(512, 256, 256, design, storage, steps=5000)


def capsule_crop(design: str = "SCS", storage: str = "f32") -> Case:
    return capsule_swimmer(128, 64, 64, design, storage, steps=1000)


def batched_sweep(seed: int = 7, n: int = 96, periods: int = 10, storage: str = "f32") -> List[Case]:
    """96 independent C1-type swimmers with per-swimmer draws, in this order:
    (nx, ny, nz, tau, amplitude, period, phase lag).  Boxes with tau below
    0.7 move their bodies with the two-step mean of the hydrodynamic force:
    under the plain explicit coupling every box of this sweep with
    tau <= 0.668 grows a step-to-step oscillation of the body velocities
    within 4000 steps, and none with tau >= 0.679 does.  The others keep
    the plain coupling of Alg. 2."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(n):
        nx = int(rng.choice([96, 128, 160]))
        ny = int(rng.choice([48, 64]))
        nz = int(rng.choice([48, 64]))
        tau = float(rng.uniform(0.6, 1.2))
        a = float(rng.uniform(1e-4, 5e-4))
        T = int(rng.choice([400, 800, 1200]))
        psi = float(rng.uniform(0.0, math.pi))
        b, s, d = swimmer((nx / 2.0, ny / 2.0, nz / 2.0), r=3.0, l0=(10.0, 10.0), k=0.05,
                          gamma=0.01, amplitude=a, period=float(T), phase_lag=psi)
        out.append(Case(f"sweep{q:02d}_{nx}x{ny}x{nz}", nx, ny, nz, tau, bodies=b, springs=s,
                        drives=[d], steps=periods * T, storage=storage, force_average=tau < 0.7))
    return out


def adjoint_case(storage: str = "f32", periods: int = 2) -> Case:
    """128x64x64, tau 0.9, r=4 swimmer, l0=16, period 500, two periods."""
    b, s, d = swimmer((64.0, 32.0, 32.0), r=4.0, l0=(16.0, 16.0), k=0.05, gamma=0.01,
                      amplitude=2e-4, period=500.0, phase_lag=math.pi / 2)
    return Case("adjoint_128x64x64", 128, 64, 64, 0.9, bodies=b, springs=s, drives=[d],
                steps=periods * 500, storage=storage)


# --------------------------------------------------------------------------
# Test workloads
# --------------------------------------------------------------------------

def forced_motion(steps: int = 400, storage: str = "f64") -> Case:
    """A kinematic sphere (r=4) dragged at V=(0.031, 0.017, 0) lu/step through a
    64x48x48 channel: it crosses about a dozen cells, so cells are covered and
    uncovered (refilled) throughout the run."""
    body = make_body(SPHERE, 4.0, bead_mass(4.0), (20.0, 17.0, 24.0),
                     vel=(0.031, 0.017, 0.0), kinematic=True)
    return Case("forced_motion_64x48x48", 64, 48, 48, 0.8, bodies=[body], steps=steps,
                storage=storage)


# Sec. 5.1 design study, converted to lattice units: dx = 1 um, the time step
# fixed by the printed driving frequency (omega = 296057.86703 1/s for a
# period of 28116 steps), fluid density 1360 kg/m^3 (the printed 1.36 read
# with the unit of g/cm^3).
PAPER_SI = {"dx": 1e-6, "omega": 296057.86703, "period": 28116, "rho": 1360.0, "mass": 5.44e-13,
            "k": 1.72965, "gamma": 1.57237e-7, "amplitude": 1.0e-5}


def paper_units():
    """Lattice values of the Sec. 5.1 parameters: (mass, k, gamma, amplitude)."""
    si = PAPER_SI
    dt = (2.0 * math.pi / si["period"]) / si["omega"]
    mu = si["rho"] * si["dx"] ** 3                  # mass unit
    return (si["mass"] / mu, si["k"] * dt * dt / mu, si["gamma"] * dt / mu,
            si["amplitude"] * dt * dt / (mu * si["dx"]))


# The Sec. 5.1 design table: bodies (left, middle, right), S a sphere and C a
# capsule, and the capsules' axis: along the swimmer axis (x) or across it
# (y).  Which body carries the capsule follows from the printed total
# lengths, GA factors and per-body Reynolds numbers; for the designs with one
# capsule at an end it follows from the printed arm amplitudes, the arm next
# to a capsule oscillating less.
PAPER_DESIGNS = {
    "a": ("SSS", None), "q": ("SSS", None),
    "b": ("CSS", "x"), "c": ("SCS", "x"), "d": ("SSC", "x"), "e": ("CSC", "x"), "f": ("CCC", "x"),
    "g": ("CSS", "y"), "h": ("SCS", "y"), "i": ("SSC", "y"), "j": ("CSC", "y"), "k": ("CCC", "y"),
    "l": ("CSS", "y"), "m": ("SCS", "y"), "n": ("SSC", "y"), "o": ("CSC", "y"), "p": ("CCC", "y"),
}


def paper_rest_gap(design: str, a: str, b: str) -> float:
    """Surface gap of the spring between bodies of kinds ``a`` and ``b``: 8
    cells, except in the long perpendicular family (g)-(k), where it is 12
    between a sphere and a capsule and 16 between two capsules, so that those
    arms are as long as in the parallel family (b)-(f)."""
    if design in "ghijk":
        return 8.0 + 4.0 * ((a == "C") + (b == "C"))
    return 8.0


def paper_design(design: str = "a", storage: str = "f64") -> Case:
    """A swimmer of the Sec. 5.1 design study, centred in a 200x100x100
    channel (swimmer axis x, periodic; walls in y and z), tau 2/3.

    Spheres of radius 4 ((q): radius 8), capsules of radius 4 and length 16
    (cylinder 8); every body has the same mass.  Spring rest lengths are
    surface gaps (``paper_rest_gap``) plus the bodies' half extents along x.
    The right force starts a quarter period late; the forces are switched off
    after five periods (left) and a quarter period later (right and middle);
    196812 steps in all.  Capsules do not rotate.  The bodies move with the
    two-step mean of the hydrodynamic force: at tau = 2/3 the plain explicit
    coupling lets a period-2 oscillation grow until the swimmer is torn
    apart."""
    kinds, axis = PAPER_DESIGNS[design]
    r, h = (8.0 if design == "q" else 4.0), 4.0
    m, k, gamma, a = paper_units()
    T = PAPER_SI["period"]

    def half(kind):
        return r + h if (kind == "C" and axis == "x") else r

    left, middle, right = kinds
    l0 = (paper_rest_gap(design, left, middle) + half(left) + half(middle),
          paper_rest_gap(design, middle, right) + half(middle) + half(right))
    shapes = tuple(CAPSULE if c == "C" else SPHERE for c in (middle, left, right))
    b, s, d = swimmer((100.0, 50.0, 50.0), shapes=shapes, r=r, h=h, l0=l0, k=k, gamma=gamma, mass=m,
                      amplitude=a, period=float(T), phase_lag=math.pi / 2, gate_lagged=True,
                      off_left=5 * T, off_right=5 * T + T // 4)
    c45 = math.sqrt(0.5)
    for body in b:
        if body.shape == CAPSULE:
            body.kinematic = 2
            if axis == "y":
                body.quat = (c45, 0.0, 0.0, c45)   # body x axis turned onto y
    return Case(f"paper_{design}_200x100x100", 200, 100, 100, 2.0 / 3.0, bodies=b, springs=s, drives=[d],
                steps=196812, storage=storage, force_average=True)


def paper_flow_channel(swimmers: int = 3, storage: str = "f32") -> Case:
    """The channel of the averaged flow fields of Sec. 6 (Fig. flowfields13):
    164x164 cells across, 240 along the swimmer axis (x here, periodic),
    with the parameters of the design study; one or three swimmers of
    design (a), driven alike.  The figure alone shows where the three swim;
    the reading here puts them side by side across the channel, 32 cells
    apart along y, all centred in z and in x (a plane of mirror symmetry at
    the middle swimmer, and one through all three)."""
    one = paper_design("a", storage)
    bodies, springs, drives = [], [], []
    offsets = (0.0,) if swimmers == 1 else (-32.0, 0.0, 32.0)
    if swimmers not in (1, 3):
        raise ValueError("one or three swimmers")
    for s_, dy in enumerate(offsets):
        base = 3 * s_
        for b in one.bodies:
            bodies.append(dataclasses.replace(b, anchor=(b.anchor[0] + 20.0, 82.0 + dy, 82.0)))
        springs += [dataclasses.replace(sp, i=sp.i + base, j=sp.j + base) for sp in one.springs]
        d = one.drives[0]
        drives.append(dataclasses.replace(d, left=d.left + base, middle=d.middle + base, right=d.right + base))
    return Case(f"paper_flow_{swimmers}_240x164x164", 240, 164, 164, one.tau, bodies=bodies, springs=springs,
                drives=drives, steps=one.steps, storage=storage, force_average=True)


# Sec. 4: range of the spring constant in the resonance sweep (kg/s^2)
VACUUM_K_RANGE = (4.76813e-3, 0.181309)


def vacuum_sweep(n: int = 38, steps: int = 1_000_000, amplitude: float = 1e-6) -> List[Case]:
    """The integrator-only runs of Sec. 4 (Fig. vacuumVal2): the three-sphere
    swimmer in vacuum with the left, middle and right spheres at x = 25, 50,
    75 and rest lengths 25, the lattice mass 400 of the design study, the
    driving period T = 28116 with the right force delayed by T/4 (ungated and
    never switched off, so that the drive is a pure sinusoid) and the damping
    ratio D = 0.07 of Eq. dampingFactor in every run.  The n spring
    constants put omega_0 / omega = sqrt(k / m) / omega evenly over the
    printed range of k (0.316 ... 1.950).  The box is nominal: no fluid.

    The drive amplitude of these runs is not given.  At the design study's
    a = 4.19e-3 the softest springs would stretch by up to about 2000 cells
    and the bodies would pass through one another, outside the linear model
    of Sec. 4; the amplitude plotted, A / a, does not depend on a while the
    motion stays linear, so a = 1e-6 keeps every arm within a cell of its
    rest length."""
    m, k_paper, _, _ = paper_units()
    a = amplitude
    T = PAPER_SI["period"]
    w = 2.0 * math.pi / T
    per_si = k_paper / PAPER_SI["k"]          # lattice stiffness per kg/s^2
    lo, hi = (math.sqrt(k * per_si / m) / w for k in VACUUM_K_RANGE)
    cases = []
    for ratio in np.linspace(lo, hi, n):
        k = m * (ratio * w) ** 2
        gamma = 2.0 * 0.07 * math.sqrt(m * k)
        b, s, d = swimmer((50.0, 50.0, 50.0), r=4.0, l0=(25.0, 25.0), k=k, gamma=gamma, mass=m, amplitude=a,
                          period=float(T), phase_lag=math.pi / 2)
        cases.append(Case(f"vacuum_w0_{ratio:.4f}", 100, 100, 100, 1.0, bodies=b, springs=s, drives=[d],
                          steps=steps))
    return cases


def vacuum_position_plot() -> Case:
    """The vacuum run of Fig. positionPlot (Sec. 4): the design study's
    masses, springs and driving (gated right force, switched off at 5T and
    5T + T/4) on spheres at x = 25, 50, 75 with rest lengths 25, for the
    196812 steps of the caption.  The box is nominal: no fluid."""
    m, k, gamma, a = paper_units()
    T = PAPER_SI["period"]
    b, s, d = swimmer((50.0, 50.0, 50.0), r=4.0, l0=(25.0, 25.0), k=k, gamma=gamma, mass=m, amplitude=a,
                      period=float(T), phase_lag=math.pi / 2, gate_lagged=True, off_left=5 * T,
                      off_right=5 * T + T // 4)
    return Case("vacuum_position_plot", 100, 100, 100, 1.0, bodies=b, springs=s, drives=[d], steps=196812)


def random_small(seed: int, storage: str = "f64") -> Case:
    """A small random box with one to three free, kinematic or rotation-locked
    spheres/capsules,
    placed without overlap and away from the walls; used for property tests."""
    rng = np.random.default_rng(1000 + seed)
    nx = int(rng.integers(12, 29))
    ny = int(rng.integers(12, 25))
    nz = int(rng.integers(12, 25))
    periodic = (True, bool(rng.integers(0, 2)), False)
    tau = float(rng.uniform(0.55, 1.6))
    nb = int(rng.integers(1, 4))
    bodies: List[Body] = []
    tries = 0
    while len(bodies) < nb and tries < 200:
        tries += 1
        shape = int(rng.integers(0, 2))
        r = float(rng.uniform(1.2, 3.0))
        h = float(rng.uniform(0.5, 2.5)) if shape == CAPSULE else 0.0
        ext = r + h
        lo = [ext + 1.5] * 3
        hi = [nx - ext - 1.5, ny - ext - 1.5, nz - ext - 1.5]
        if any(h_ <= l_ for l_, h_ in zip(lo, hi)):
            continue
        pos = [float(rng.uniform(l_, h_)) for l_, h_ in zip(lo, hi)]
        ok = True
        for other in bodies:
            d = math.dist(pos, other.anchor)
            if d < ext + other.radius + other.half_len + 2.5:
                ok = False
        if not ok:
            continue
        kin = int(rng.integers(0, 3))   # free, prescribed motion, rotation locked
        vel = tuple(float(v) for v in rng.uniform(-0.02, 0.02, 3)) if kin == 1 else (0.0, 0.0, 0.0)
        omg = tuple(float(v) for v in rng.uniform(-0.01, 0.01, 3)) if kin else (0.0, 0.0, 0.0)
        ang = float(rng.uniform(0, math.pi))
        ax = rng.normal(size=3)
        ax = ax / np.linalg.norm(ax)
        quat = (math.cos(ang / 2),) + tuple(float(v) * math.sin(ang / 2) for v in ax)
        # every body at the spheres' density ratio (about 1.49): a free capsule
        # of the spheres' mass would be lighter than the fluid, and its
        # rotation unstable under the explicit coupling
        m = bead_mass(r) * (1.0 + 1.5 * h / r)
        b = make_body(shape, r, m, pos, h, vel=vel, omega=omg, quat=quat, kinematic=kin)
        bodies.append(b)
    springs: List[Spring] = []
    drives: List[Drive] = []
    if len(bodies) == 3:
        springs = [Spring(1, 0, 0.05, 0.01, math.dist(bodies[1].anchor, bodies[0].anchor)),
                   Spring(2, 0, 0.05, 0.01, math.dist(bodies[2].anchor, bodies[0].anchor))]
        drives = [Drive(1, 0, 2, 1e-3, 40.0, float(rng.uniform(0, math.pi)))]
    return Case(f"random{seed}_{nx}x{ny}x{nz}", nx, ny, nz, tau, periodic=periodic,
                bodies=bodies, springs=springs, drives=drives, steps=int(rng.integers(8, 30)),
                storage=storage)


def initial_populations(case: Case, seed: int, amp: float = 1e-3) -> np.ndarray:
    """Seeded random deviations dF (shape [19, nz, ny, nx], float64) for tests that
    start from a perturbed state; bodies' cells are left as given (the method
    discards populations inside bodies)."""
    rng = np.random.default_rng(seed)
    return amp * rng.standard_normal((19, case.nz, case.ny, case.nx))
