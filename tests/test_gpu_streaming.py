"""In-place streaming (LBM_TUNE_STREAMING = 1, the AA access pattern) on the
GPU through the C-ABI.

The in-place sweep does the arithmetic of the two-buffer sweep (Eq. lbgk,
Eq. streaming, the moving bounce-back and momentum exchange of Sec. 2.3);
only where each population sits between steps differs, and the exports read
through the layout.  So the two modes must agree bit for bit: populations,
trajectories (force, torque, displacement of every step) and flags, over runs
whose bodies cross cells at even and at odd steps (the remap in the swapped
layout moves populations between slots), in every storage format, with one
or all of a box's workgroups mapping, in batches whose boxes stop at
different steps (so that their parities differ), when the mode is switched
in the middle of a run at an odd step, and around the adjoint (which runs the
two-buffer sweep on a converted copy).  The oracle pins the in-place mode
directly on the swimmer case and on the forced motion: 1e-12 in FP64."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import OracleSim

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _sim(case, **kw):
    from paper_1108_0786_amd.sim import Sim
    return Sim(case, device="cuda:0", **kw)


def _rel(a, b):
    scale = np.abs(b).max()
    return np.abs(a - b).max() / scale if scale > 0 else np.abs(a - b).max()


def _same(a, b, steps):
    assert np.array_equal(a.populations(), b.populations()), "populations differ"
    assert np.array_equal(a.trajectory()[:steps], b.trajectory()[:steps]), "trajectories differ"
    assert np.array_equal(a.flags(), b.flags()), "flags differ"


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "bf16s"])
@pytest.mark.parametrize("coop", [0, 1, 2])
def test_in_place_matches_two_buffer_bitwise(storage, coop):
    # a kinematic sphere dragged across about a dozen cells: cells change
    # side at even and at odd steps
    steps = 160
    case = W.forced_motion(steps=steps, storage=storage)
    print(f"[gpu] in-place vs two-buffer, {storage}, coop {coop}", flush=True)
    ref = _sim(case, storage=storage, traj_cap=steps, tune={"coop_remap": coop, "streaming": 0})
    aa = _sim(case, storage=storage, traj_cap=steps, tune={"coop_remap": coop, "streaming": 1})
    flags0 = aa.flags()
    odd_changes = even_changes = 0
    for n in range(steps):
        ref.step(1)
        aa.step(1)
        f = aa.flags()
        if not np.array_equal(f & 0x7F, flags0 & 0x7F):
            # the remap after step n sees the layout of step n + 1
            if (n + 1) % 2:
                odd_changes += 1
            else:
                even_changes += 1
        flags0 = f
    assert odd_changes > 2 and even_changes > 2, (odd_changes, even_changes)
    _same(ref, aa, steps)
    ref.close()
    aa.close()


def test_in_place_forced_motion_against_oracle():
    steps = 120
    case = W.forced_motion(steps=steps)
    df0 = W.initial_populations(case, seed=5, amp=1e-4)
    print("[gpu] in-place forced motion vs oracle", flush=True)
    orc = OracleSim(case, df0=df0).run(steps)
    aa = _sim(case, storage="f64", traj_cap=steps, df0=df0, tune={"streaming": 1})
    aa.step(steps)
    aa.status()
    orc.map_next()              # the library maps step n + 1 at the end of step n
    assert np.array_equal(aa.flags() & 0x7F, orc.flags)
    assert _rel(aa.populations(), orc.populations()) < 1e-12
    F = aa.trajectory()[:steps, :, 9:12]
    Fo = np.array([t["F"] for t in orc.traj], dtype=float)
    assert _rel(F, Fo) < 1e-12
    aa.close()


def test_in_place_swimmer_against_oracle():
    case = W.plain_f64_small()
    steps = 61                                      # ends in the swapped layout
    print("[gpu] in-place swimmer vs oracle", flush=True)
    orc = OracleSim(case).run(steps)
    aa = _sim(case, storage="f64", traj_cap=steps, tune={"streaming": 1})
    aa.step(steps)
    orc.map_next()
    assert _rel(aa.populations(), orc.populations()) < 1e-12
    D = aa.trajectory()[:steps, :, 0:3]
    Do = np.array([t["D"] for t in orc.traj], dtype=float)
    assert _rel(D, Do) < 1e-12
    aa.close()


def test_switching_mode_mid_run():
    # two-buffer for 7 steps, in place from the odd step 7 to 20, two-buffer
    # again from the odd step 21: the same run as two-buffer throughout
    steps = 33
    case = W.forced_motion(steps=steps)
    print("[gpu] streaming mode switched mid-run", flush=True)
    ref = _sim(case, storage="f64", traj_cap=steps, tune={"streaming": 0})
    ref.step(steps)
    sw = _sim(case, storage="f64", traj_cap=steps, tune={"streaming": 0})
    sw.step(7)
    sw.tune("streaming", 1)
    sw.step(14)
    sw.tune("streaming", 0)
    sw.step(12)
    _same(ref, sw, steps)
    ref.close()
    sw.close()


def test_imports_and_exports_through_the_layout():
    # populations imported at an odd step (swapped layout) come back unchanged
    case = W.forced_motion(steps=10)
    aa = _sim(case, storage="f64", tune={"streaming": 1})
    aa.step(3)
    df = aa.populations()
    rng = np.random.default_rng(4)
    new = df + 1e-5 * rng.standard_normal(df.shape) * (df != 0)
    aa.import_populations(new)
    assert np.array_equal(aa.populations(), new)
    cells = np.array([0, 17, 1000, aa.flags().size - 1], dtype=np.int32)
    at = aa.populations_at(cells)
    assert np.array_equal(at, new.reshape(19, -1)[:, cells])
    aa.close()


def test_batched_boxes_at_different_parities():
    from paper_1108_0786_amd.sim import BatchSim
    cases = [W.forced_motion(steps=40), W.plain_f64_small(), W.forced_motion(steps=40)]
    limits = [40, 37, 29]
    print("[gpu] in-place batch with step limits", flush=True)
    out = []
    for streaming in (0, 1):
        b = BatchSim(cases, storage="f64", traj_cap=40, tune={"streaming": streaming})
        for i, n in enumerate(limits):
            b.set_step_limit(i, n)
        b.step(40)
        out.append([(b.populations(i), b.trajectory(i)[:limits[i]], b.flags(i)) for i in range(len(cases))])
        b.close()
    for (p0, t0, f0), (p1, t1, f1) in zip(*out):
        assert np.array_equal(p0, p1) and np.array_equal(t0, t1) and np.array_equal(f0, f1)


def test_adjoint_is_the_same_in_either_mode():
    b, s, d = W.swimmer((20.0, 12.0, 12.0), r=3.0, l0=(8.0, 8.0), k=0.05, gamma=0.01,
                        amplitude=2e-4, period=40.0, phase_lag=math.pi / 2)
    case = W.Case("adjoint_small", 40, 24, 24, 0.9, bodies=b, springs=s, drives=[d], steps=40)
    print("[gpu] adjoint in both streaming modes", flush=True)
    res = []
    for streaming in (0, 1):
        sim = _sim(case, storage="f64", tune={"streaming": streaming})
        sim.step(3)                                  # start at an odd step
        J, g = sim.adjoint(33, 8)
        sim.step(2)
        res.append((J, g, sim.populations(), sim.bodies()))
        sim.close()
    assert res[0][0] == res[1][0]
    assert np.array_equal(res[0][1], res[1][1])
    assert np.array_equal(res[0][2], res[1][2])
    assert [x["D"] for x in res[0][3]] == [x["D"] for x in res[1][3]]
