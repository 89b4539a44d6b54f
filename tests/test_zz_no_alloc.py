"""``lbm_vacuum_run_noalloc``, the integrator-only run for callers that cannot
allocate device memory, against ``lbm_vacuum_run`` through the C-ABI.  Both
run the same kernel on the same tables, so final states and trajectories are
compared bit for bit: on two calls in a row, the second with fewer systems
and steps than the first (the array the first call filled keeps its
contents), and once more after a call whose tables do not fit has been
turned away."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _states(states):
    return np.array([[np.concatenate([b["D"], b["V"], b["quat"], b["Omega"]]) for b in s] for s in states])


def _same_run(cases, steps, traj_cap):
    from paper_1108_0786_amd.sim import vacuum_run
    print(f"[gpu] no-alloc vacuum run: {len(cases)} systems, {steps} steps", flush=True)
    s_ref, t_ref = vacuum_run(cases, steps, traj_cap=traj_cap)
    s_new, t_new = vacuum_run(cases, steps, traj_cap=traj_cap, noalloc=True)
    assert np.array_equal(_states(s_ref), _states(s_new))
    assert np.array_equal(t_ref, t_new)
    assert np.abs(_states(s_new)[:, :, 0]).max() > 0      # the drive moved the bodies


def _oversize(n):
    """n copies of one three-bead system through the C-ABI, no trajectory."""
    from paper_1108_0786_amd import _abi
    from paper_1108_0786_amd.sim import LbmBody, LbmDrive, LbmSpring, _body_struct
    lib = _abi.load()
    c = W.vacuum_sweep(n=1, steps=10)[0]
    bodies = (LbmBody * (3 * n))(*[_body_struct(b) for _ in range(n) for b in c.bodies])
    springs = (LbmSpring * (2 * n))(*[LbmSpring(s.i, s.j, s.k, s.gamma, s.rest_len)
                                      for _ in range(n) for s in c.springs])
    d = c.drives[0]
    drives = (LbmDrive * n)(*[LbmDrive(d.left, d.middle, d.right, int(d.gate_lagged), d.amplitude, d.period,
                                       d.phase_lag, d.off_left, d.off_right) for _ in range(n)])
    out = (LbmBody * (3 * n))()
    return lib.lbm_vacuum_run_noalloc(bodies, 3, springs, 2, drives, 1, n, 10, None, 0, out, None)


def test_no_alloc_run_matches_allocating_run():
    from paper_1108_0786_amd import _abi
    sweep = W.vacuum_sweep(n=38)
    _same_run(sweep[::2], 3000, traj_cap=64)              # 19 systems
    _same_run(sweep[5:9], 1200, traj_cap=16)              # fewer systems, fewer steps
    print("[gpu] no-alloc: oversize rejected", flush=True)
    assert _oversize(1000) == _abi.LBM_E_ARG               # 1000 systems need about 1.2 MB
    _same_run(sweep[1:2], 500, traj_cap=0)
