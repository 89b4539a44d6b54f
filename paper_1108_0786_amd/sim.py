"""Python binding of the swimmer step: torch supplies device memory and the
stream, every step of the method runs in the library's HIP kernels.

``Sim`` wraps one box (lbm_init); ``BatchSim`` wraps many independent boxes
stepped together by single launches (lbm_init_batch)."""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _abi
from ._abi import LbmBody, LbmDrive, LbmParams, LbmSpring, check

_TORCH_DTYPE = {"f64": torch.float64, "f32": torch.float32, "f16s": torch.float16, "bf16s": torch.bfloat16}


def _body_struct(b):
    s = LbmBody()
    s.shape = int(b.shape)
    s.kinematic = int(b.kinematic)
    s.radius = float(b.radius)
    s.half_len = float(b.half_len)
    s.mass = float(b.mass)
    for q in range(3):
        s.inertia[q] = float(b.inertia[q])
        s.anchor[q] = float(b.anchor[q])
        s.disp[q] = float(b.disp[q])
        s.vel[q] = float(b.vel[q])
        s.omega[q] = float(b.omega[q])
    for q in range(4):
        s.quat[q] = float(b.quat[q])
    return s


def _arrays(case):
    nb, ns, nd = len(case.bodies), len(case.springs), len(case.drives)
    bodies = (LbmBody * max(nb, 1))(*[_body_struct(b) for b in case.bodies])
    springs = (LbmSpring * max(ns, 1))(*[LbmSpring(s.i, s.j, s.k, s.gamma, s.rest_len) for s in case.springs])
    drives = (LbmDrive * max(nd, 1))(*[LbmDrive(d.left, d.middle, d.right, int(d.gate_lagged), d.amplitude,
                                                d.period, d.phase_lag, d.off_left, d.off_right)
                                       for d in case.drives])
    return bodies, nb, springs, ns, drives, nd


def _body_dict(s):
    return {"shape": s.shape, "kinematic": int(s.kinematic), "radius": s.radius, "half_len": s.half_len,
            "mass": s.mass, "anchor": list(s.anchor), "D": list(s.disp), "quat": list(s.quat),
            "V": list(s.vel), "Omega": list(s.omega)}


def padded_stride(n, pad=None):
    """Elements between consecutive directions' arrays: N rounded up to 256
    elements plus ``pad`` (default 1024), so that the 19 streams of a sweep do
    not sit at a power-of-two spacing in HBM.  On the 256x128x128 box any pad
    from 512 to 3072 elements gives the same sweep time within 1%; 1024 is 2%
    (FP32) and 4% (FP64) faster than 4160 and the same for the 16-bit
    formats."""
    if pad is None:
        pad = DEFAULT_PAD
    return (n + 255) // 256 * 256 + pad if pad else n


DEFAULT_PAD = 1024


class _Box:
    """Device buffers of one box (caller-owned memory of the C-ABI)."""

    def __init__(self, case, storage, device, traj_cap, shift_log2, pad=None, body_force=None):
        self.case = case
        self.N = case.nx * case.ny * case.nz
        self.stride = padded_stride(self.N, pad)
        dt = _TORCH_DTYPE[storage]
        self.pop = [torch.zeros(19 * self.stride, dtype=dt, device=device) for _ in range(2)]
        self.flags = torch.zeros(self.N, dtype=torch.uint8, device=device)
        nb = max(len(case.bodies), 1)
        self.traj = torch.zeros((traj_cap, nb, _abi.TRAJ_DOUBLES), dtype=torch.float64,
                                device=device) if traj_cap else None
        p = LbmParams()
        p.nx, p.ny, p.nz = case.nx, case.ny, case.nz
        p.periodic_mask = sum(1 << q for q in range(3) if case.periodic[q])
        p.tau = float(case.tau)
        p.storage = _abi.STORAGE[storage]
        p.shift_log2 = int(shift_log2)
        p.pop[0] = self.pop[0].data_ptr()
        p.pop[1] = self.pop[1].data_ptr()
        p.flags = self.flags.data_ptr()
        p.traj = self.traj.data_ptr() if self.traj is not None else None
        p.traj_cap = traj_cap
        p.stream = torch.cuda.current_stream(device).cuda_stream
        p.stride = self.stride
        p.force_average = int(bool(getattr(case, "force_average", False)))
        if body_force is not None:            # test-only uniform force on the fluid
            for q in range(3):
                p.body_force[q] = float(body_force[q])
        self.params = p


class BatchSim:
    """Many independent boxes, each with its own swimmer, in one context."""

    def __init__(self, cases, storage=None, device="cuda:0", traj_cap=0, shift_log2=None, df0=None,
                 pad=None, tune=None, body_force=None):
        self.lib = _abi.load()
        self.device = torch.device(device)
        storage = storage or cases[0].storage
        self.storage = storage
        if shift_log2 is None:
            shift_log2 = cases[0].shift_log2 if storage in ("f16s", "bf16s") else 0
        with torch.cuda.device(self.device):
            self.boxes = [_Box(c, storage, self.device, traj_cap, shift_log2, pad, body_force) for c in cases]
            arr = (LbmParams * len(cases))(*[b.params for b in self.boxes])
            self.ctx = C.c_void_p()
            rc = self.lib.lbm_init_batch(arr, len(cases), C.byref(self.ctx))
            if rc != 0:
                err = _abi.LbmError(rc, (self.lib.lbm_last_error(self.ctx) or b"").decode())
                self.lib.lbm_destroy(self.ctx)
                self.ctx = None
                raise err
            for key, val in (tune or {}).items():
                self.tune(key, val)
            if df0 is not None:
                for i, d in enumerate(df0):
                    if d is not None:
                        self.import_populations(d, i)
            for i, c in enumerate(cases):
                self.set_bodies(c, i)

    # -- calls of the C-ABI ------------------------------------------------
    def set_bodies(self, case, box=0):
        bodies, nb, springs, ns, drives, nd = _arrays(case)
        check(self.lib, self.ctx, self.lib.lbm_set_bodies_box(self.ctx, box, bodies, nb, springs, ns, drives, nd))

    def tune(self, key, value):
        check(self.lib, self.ctx, self.lib.lbm_tune(self.ctx, _abi.TUNE[key], int(value)))

    def set_step_limit(self, box, steps):
        check(self.lib, self.ctx, self.lib.lbm_set_step_limit(self.ctx, box, int(steps)))

    def step(self, n=1):
        check(self.lib, self.ctx, self.lib.lbm_step(self.ctx, int(n)))

    def prepare(self, n):
        """Capture the graphs that step(n) replays, without running them."""
        check(self.lib, self.ctx, self.lib.lbm_prepare(self.ctx, int(n)))

    def status(self):
        return check(self.lib, self.ctx, self.lib.lbm_status(self.ctx))

    def forces(self, box=0):
        nb = len(self.boxes[box].case.bodies)
        F = np.zeros((nb, 3))
        T = np.zeros((nb, 3))
        check(self.lib, self.ctx, self.lib.lbm_body_forces_box(
            self.ctx, box, F.ctypes.data_as(C.c_void_p), T.ctypes.data_as(C.c_void_p), 0))
        return F, T

    def bodies(self, box=0):
        nb = len(self.boxes[box].case.bodies)
        out = (LbmBody * max(nb, 1))()
        check(self.lib, self.ctx, self.lib.lbm_get_bodies_box(self.ctx, box, out, nb))
        return [_body_dict(out[b]) for b in range(nb)]

    def links(self, box=0):
        n = C.c_int64()
        cap = 18 * self.boxes[box].N
        rc = self.lib.lbm_get_links(self.ctx, box, None, None, None, 0, C.byref(n))
        if rc not in (0, _abi.LBM_E_CAPACITY):
            check(self.lib, self.ctx, rc)
        cell = np.zeros(max(n.value, 1), np.int32)
        d = np.zeros(max(n.value, 1), np.int8)
        b = np.zeros(max(n.value, 1), np.int8)
        check(self.lib, self.ctx, self.lib.lbm_get_links(
            self.ctx, box, cell.ctypes.data_as(C.c_void_p), d.ctypes.data_as(C.c_void_p),
            b.ctypes.data_as(C.c_void_p), min(cap, n.value), C.byref(n)))
        k = n.value
        return cell[:k].astype(np.int64), d[:k].astype(np.int64), b[:k].astype(np.int64)

    def populations(self, box=0):
        """Current deviations dF as float64 numpy (19, nz, ny, nx); zero in bodies."""
        bx = self.boxes[box]
        out = torch.empty(19 * bx.N, dtype=torch.float64, device=self.device)
        check(self.lib, self.ctx, self.lib.lbm_export_populations(self.ctx, box, C.c_void_p(out.data_ptr())))
        c = bx.case
        return out.cpu().numpy().reshape(19, c.nz, c.ny, c.nx)

    def populations_at(self, cells, box=0):
        """Current deviations at the given linear cell indices, float64 numpy (19, n)."""
        idx = torch.as_tensor(np.ascontiguousarray(cells, dtype=np.int32)).to(self.device)
        n = idx.numel()
        out = torch.empty(19 * max(n, 1), dtype=torch.float64, device=self.device)
        check(self.lib, self.ctx, self.lib.lbm_export_cells(self.ctx, box, C.c_void_p(idx.data_ptr()), n,
                                                             C.c_void_p(out.data_ptr())))
        return out[:19 * n].cpu().numpy().reshape(19, n)

    def import_populations(self, df, box=0):
        bx = self.boxes[box]
        t = torch.as_tensor(np.ascontiguousarray(df, dtype=np.float64).reshape(-1)).to(self.device)
        check(self.lib, self.ctx, self.lib.lbm_import_populations(self.ctx, box, C.c_void_p(t.data_ptr())))
        torch.cuda.synchronize(self.device)

    def flow_average_begin(self, every, box=0):
        """Start (every >= 1, clearing the sums) or stop (every = 0) sampling
        the time-averaged fluid velocity of a box."""
        check(self.lib, self.ctx, self.lib.lbm_flow_average_begin(self.ctx, box, int(every)))

    def flow_average(self, box=0):
        """(mean velocity (3, nz, ny, nx), sample counts (nz, ny, nx)) as numpy."""
        bx = self.boxes[box]
        c = bx.case
        mean = torch.empty(3 * bx.N, dtype=torch.float64, device=self.device)
        cnt = torch.empty(bx.N, dtype=torch.int32, device=self.device)
        check(self.lib, self.ctx, self.lib.lbm_flow_average_get(self.ctx, box, C.c_void_p(mean.data_ptr()),
                                                                C.c_void_p(cnt.data_ptr())))
        return (mean.cpu().numpy().reshape(3, c.nz, c.ny, c.nx), cnt.cpu().numpy().reshape(c.nz, c.ny, c.nx))

    def flags(self, box=0):
        return self.boxes[box].flags.cpu().numpy()

    def step_count(self, box=0):
        n = C.c_int64()
        check(self.lib, self.ctx, self.lib.lbm_step_count(self.ctx, box, C.byref(n)))
        return n.value

    def set_timing(self, enable):
        check(self.lib, self.ctx, self.lib.lbm_set_timing(self.ctx, int(bool(enable))))

    def timing(self):
        """(sweep_ms, sweep_launches, coupling_ms, coupling_launches) since timing was enabled."""
        ms = (C.c_double * 2)()
        n = (C.c_int64 * 2)()
        check(self.lib, self.ctx, self.lib.lbm_get_timing(self.ctx, ms, n))
        return ms[0], n[0], ms[1], n[1]

    def trajectory(self, box=0):
        t = self.boxes[box].traj
        return None if t is None else t.cpu().numpy()

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sim(BatchSim):
    """One box: ``Sim(case)`` maps ``case.bodies`` and is ready to step."""

    def __init__(self, case, storage=None, device="cuda:0", traj_cap=0, shift_log2=None, df0=None,
                 pad=None, tune=None, body_force=None):
        super().__init__([case], storage=storage, device=device, traj_cap=traj_cap,
                         shift_log2=shift_log2, df0=None if df0 is None else [df0], pad=pad, tune=tune,
                         body_force=body_force)

    def centroid_displacement(self):
        b = self.bodies()
        return sum(x["D"][0] for x in b) / len(b)

    def adjoint(self, steps, checkpoint_every=50, weights=None):
        """Run ``steps`` coupled steps and the hand-written reverse pass.

        J = sum_b weights[b] . disp_b at the end (default: the x displacement
        of the centroid, 1/nb on x).  Returns (J, dJ/d(amplitude, phase_lag, k))."""
        nb = len(self.boxes[0].case.bodies)
        if weights is None:
            weights = np.zeros((nb, 3))
            weights[:, 0] = 1.0 / nb
        w = np.ascontiguousarray(weights, dtype=np.float64).reshape(nb * 3)
        J = C.c_double()
        g = (C.c_double * 3)()
        check(self.lib, self.ctx, self.lib.lbm_adjoint(
            self.ctx, int(steps), int(checkpoint_every), w.ctypes.data_as(C.POINTER(C.c_double)),
            C.byref(J), g))
        return J.value, np.array(list(g))


def vacuum_run(cases, steps, traj_cap=0, device="cuda:0", noalloc=False):
    """Integrator-only runs of the swimmers of ``cases`` (one system each, all
    with the same numbers of bodies, springs and drives) for ``steps`` steps
    through ``lbm_vacuum_run`` (``lbm_vacuum_run_noalloc`` with ``noalloc``).
    Returns (final body states per system, the trajectory ring as numpy
    (systems, traj_cap, bodies, 16) or None)."""
    lib = _abi.load()
    nb, ns, nd = len(cases[0].bodies), len(cases[0].springs), len(cases[0].drives)
    if any((len(c.bodies), len(c.springs), len(c.drives)) != (nb, ns, nd) for c in cases):
        raise ValueError("every system needs the same numbers of bodies, springs and drives")
    bodies = (LbmBody * (nb * len(cases)))(*[_body_struct(b) for c in cases for b in c.bodies])
    springs = (LbmSpring * max(ns * len(cases), 1))(*[LbmSpring(s.i, s.j, s.k, s.gamma, s.rest_len)
                                                       for c in cases for s in c.springs])
    drives = (LbmDrive * max(nd * len(cases), 1))(*[LbmDrive(d.left, d.middle, d.right, int(d.gate_lagged),
                                                             d.amplitude, d.period, d.phase_lag, d.off_left,
                                                             d.off_right) for c in cases for d in c.drives])
    out = (LbmBody * (nb * len(cases)))()
    dev = torch.device(device)
    traj = torch.zeros((len(cases), traj_cap, nb, _abi.TRAJ_DOUBLES), dtype=torch.float64,
                       device=dev) if traj_cap else None
    with torch.cuda.device(dev):
        stream = torch.cuda.current_stream(dev).cuda_stream
        run = lib.lbm_vacuum_run_noalloc if noalloc else lib.lbm_vacuum_run
        rc = run(bodies, nb, springs, ns, drives, nd, len(cases), int(steps),
                 C.c_void_p(traj.data_ptr()) if traj is not None else None, int(traj_cap), out, C.c_void_p(stream))
    if rc != _abi.LBM_OK:
        raise _abi.LbmError(rc, f"{run.__name__} failed")
    states = [[_body_dict(out[s * nb + b]) for b in range(nb)] for s in range(len(cases))]
    return states, (traj.cpu().numpy() if traj is not None else None)
