"""Time-averaged flow fields (Sec. 6, Fig. flowfields13) on the GPU through
the C-ABI.

Parity: the averaged fluid velocity and the per-cell sample counts against
the oracle's, element by element, on a swimmer box and on a box whose body
crosses cells (so that the set of fluid cells changes between samples).
Counts must agree bit for bit, means to 1e-12 of their largest magnitude in
FP64 storage.  Sampling must not change the run.

Paper scale: the channel of Fig. flowfields13 (164x164 across, 240 along the
axis) with three swimmers of design (a) side by side and with one, for the
paper's 196812 steps, averaged over the five driven cycles.  The paper quotes
60.28 CPU-hours for the three-swimmer run; the test prints the time here.
Asserted: stable runs, counts equal to the number of samples wherever no
body came, and the mirror symmetries of the set-ups in the averaged field
(the one-swimmer field also under the quarter turn about the axis)."""
import math
import time

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
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("name", ["swimmer", "crossing body"])
def test_flow_average_fp64_parity(name):
    case = W.plain_f64_small() if name == "swimmer" else W.forced_motion(steps=80)
    df0 = W.initial_populations(case, seed=5, amp=1e-4)
    print(f"[gpu] flow average parity {case.name}", flush=True)
    orc = OracleSim(case, df0=df0)
    sim = _sim(case, storage="f64", df0=df0)
    # every step for 30 steps, then a new average of every third step for 40
    for every, steps in ((1, 30), (3, 40)):
        orc.flow_average_begin(every)
        sim.flow_average_begin(every)
        orc.run(steps)
        sim.step(steps)
        sim.status()
        mo, co = orc.flow_average()
        mg, cg = sim.flow_average()
        samples = len([n for n in range(orc.n - steps, orc.n) if n % every == 0])
        err = _rel(mg, mo)
        print(f"[gpu] every {every}: mean err {err:.2e}, counts {cg.min()}..{cg.max()} of {samples}", flush=True)
        assert np.array_equal(cg, co)
        assert err < 1e-12
        assert cg.max() == samples
        if name == "crossing body":
            assert np.any((cg > 0) & (cg < samples))   # cells that were covered or uncovered meanwhile
    sim.close()


def test_flow_sampling_leaves_the_run_unchanged():
    case = W.forced_motion(steps=60)
    print("[gpu] flow sampling is passive", flush=True)
    ref = _sim(case, storage="f32", traj_cap=60)
    ref.step(60)
    other = _sim(case, storage="f32", traj_cap=60)
    other.flow_average_begin(2)
    other.step(30)
    mid, _ = other.flow_average()
    other.flow_average_begin(0)       # stop: the sums stay as they are
    other.step(30)
    end, _ = other.flow_average()
    assert np.array_equal(mid, end)
    assert np.array_equal(ref.populations(), other.populations())
    assert np.array_equal(ref.trajectory(), other.trajectory())
    ref.close()
    other.close()


@pytest.fixture(scope="module")
def channels():
    """The two channels of Fig. flowfields13, each advanced a period at a time
    by the tests below (so that the long runs report progress)."""
    state = {}
    yield state
    for st in state.values():
        if st["sim"] is not None:
            st["sim"].close()


def _paper_state(channels, swimmers):
    from paper_1108_0786_amd.sim import Sim
    if swimmers not in channels:
        case = W.paper_flow_channel(swimmers, "f32")
        T = W.PAPER_SI["period"]
        print(f"[gpu] flow field {case.name}: {case.steps} steps FP32, average over steps 0..{5 * T - 1}",
              flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim = Sim(case, storage="f32", traj_cap=T + 1)
        sim.flow_average_begin(1)
        channels[swimmers] = dict(sim=sim, case=case, T=T, periods=0, t0=t0, seconds=None, tr=None)
    return channels[swimmers]


def _advance(st):
    """One more period: five driven ones while the average is taken, then the
    free relaxation to the paper's 196812 steps (7 periods)."""
    sim, T = st["sim"], st["T"]
    sim.step(T)
    sim.status()
    st["periods"] += 1
    if st["periods"] == 5:
        sim.flow_average_begin(0)
        tr = sim.trajectory()         # the last driven period, steps 4T - 1 .. 5T - 1
        st["tr"] = tr[np.argsort(tr[:, 0, 15])]
    if st["periods"] == st["case"].steps // T:
        torch.cuda.synchronize()
        st["seconds"] = time.perf_counter() - st["t0"]
    print(f"[gpu] flow field {st['case'].name}: period {st['periods']} done", flush=True)


def _paper_run(channels, swimmers):
    st = _paper_state(channels, swimmers)
    total = st["case"].steps // st["T"]
    while st["periods"] < total:
        _advance(st)
    if st["sim"] is not None:
        st["mean"], st["count"] = st["sim"].flow_average()
        st["sim"].close()
        st["sim"] = None
    return st["case"], st["mean"], st["count"], st["tr"], st["seconds"]


@pytest.mark.parametrize("swimmers,period", [(3, p) for p in range(1, 8)] + [(1, p) for p in range(1, 8)])
def test_paper_flow_channel_period(channels, swimmers, period):
    st = _paper_state(channels, swimmers)
    while st["periods"] < period:
        _advance(st)


def _mirror_err(mean, axis, flip_component, keep=None):
    """Largest departure of the averaged field from the mirror image across
    the channel's mid-plane normal to ``axis`` (0 z, 1 y of the [z][y][x]
    arrays), relative to the largest speed; over the cells where ``keep`` and
    its mirror image are true, if given."""
    m = np.flip(mean, axis=1 + axis).copy()
    m[flip_component] = -m[flip_component]
    d = np.abs(mean - m).max(axis=0)
    if keep is not None:
        d = d[keep & np.flip(keep, axis=axis)]
    return d.max() / np.abs(mean).max()


@pytest.mark.parametrize("swimmers", [3, 1])
def test_paper_flow_field(channels, swimmers):
    case, mean, count, tr, seconds = _paper_run(channels, swimmers)
    T = W.PAPER_SI["period"]
    cells = case.nx * case.ny * case.nz
    vmax = np.abs(mean).max()
    assert np.array_equal(tr[:, 0, 15].astype(np.int64), np.arange(4 * T - 1, 5 * T))
    u_mid = [(tr[-1, 3 * s, 0] - tr[0, 3 * s, 0]) / T for s in range(swimmers)]
    print(f"[gpu] flow field, {swimmers} swimmer(s): {seconds:.1f} s for {case.steps} steps "
          f"({cells * case.steps / seconds / 1e9:.1f} GLUPS; the paper's three-swimmer run took 60.28 CPU-hours), "
          f"max mean speed {vmax:.3e}, u_swim of each swimmer over the fifth period: "
          + ", ".join(f"{u:.4e}" for u in u_mid), flush=True)
    assert np.all(np.isfinite(mean)) and vmax > 0
    # cells no body ever reached were sampled at every one of the 5T steps
    assert count.max() == 5 * T
    assert np.count_nonzero(count == 5 * T) > 0.99 * cells
    # mirror symmetry of the set-up across the mid-planes of y and of z.
    # Where a body came, mirror-image cells can change side at different
    # steps: the link sums of mirror-image bodies round differently, and a
    # cell centre within rounding of a surface follows its own body.  Cells
    # no body reached are held to a tighter bound.
    free = count == 5 * T
    ey, ez = _mirror_err(mean, 1, 1), _mirror_err(mean, 0, 2)
    fy, fz = _mirror_err(mean, 1, 1, free), _mirror_err(mean, 0, 2, free)
    print(f"[gpu] mirror asymmetry of the mean field: y {ey:.1e}, z {ez:.1e}; "
          f"at cells no body reached: y {fy:.1e}, z {fz:.1e}", flush=True)
    assert ey < 1e-3 and ez < 1e-3
    assert fy < 1e-5 and fz < 1e-5
    if swimmers == 1:
        # a quarter turn about the swimmer axis maps the set-up onto itself:
        # (y, z) -> (z, ny - 1 - y) with (u_y, u_z) -> (u_z, -u_y)
        rot = np.empty_like(mean)
        rot[0] = np.rot90(mean[0], k=1, axes=(0, 1))
        rot[1] = np.rot90(mean[2], k=1, axes=(0, 1))
        rot[2] = -np.rot90(mean[1], k=1, axes=(0, 1))
        er = np.abs(rot - mean).max() / vmax
        print(f"[gpu] quarter-turn asymmetry: {er:.1e}", flush=True)
        assert er < 1e-3
    else:
        # the outer swimmers are mirror images of each other
        assert math.isclose(u_mid[0], u_mid[2], rel_tol=1e-3, abs_tol=1e-9)
