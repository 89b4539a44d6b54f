"""GPU path (through the C-ABI) against the CPU oracle, element by element.

Metrics (normalised because forces and displacements cross zero):
  populations   max |dF_gpu - dF_orc| / max |dF_orc| over the box
  forces        max_n ||F_gpu - F_orc||_inf / max_n ||F_orc||_inf
  torques       the same, scaled by max ||F_orc|| times the body radius
  displacement  max_n |D_gpu - D_orc| / max_n |D_orc|
Flags and boundary links must agree bit for bit.  Tolerances: 1e-12 for
FP64 storage, 1e-5 for FP32 storage."""
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


def _oracle_traj(orc):
    F = np.array([t["F"] for t in orc.traj], dtype=float)
    T = np.array([t["T"] for t in orc.traj], dtype=float)
    D = np.array([t["D"] for t in orc.traj], dtype=float)
    return F, T, D


def _gpu_traj(sim, steps):
    tr = sim.trajectory()[:steps]
    return tr[:, :, 9:12], tr[:, :, 12:15], tr[:, :, 0:3]


def _rel(a, b):
    scale = np.abs(b).max()
    return np.abs(a - b).max() / scale if scale > 0 else np.abs(a - b).max()


def _check_geometry(sim, orc):
    orc.map_next()  # the library maps step n+1 at the end of step n
    gf = sim.flags()
    assert np.array_equal(gf & 0x7F, orc.flags), "flags differ"
    lc, ld, lb = orc.links
    near = np.zeros(orc.N, dtype=bool)
    near[lc] = True
    assert np.array_equal((gf & 0x80) != 0, near), "near-body marks differ"
    g = sim.links()
    assert np.array_equal(g[0], lc) and np.array_equal(g[1], ld) and np.array_equal(g[2], lb), "links differ"


@pytest.fixture(scope="module")
def c1_oracle():
    case = W.plain_f64_small()
    orc = OracleSim(case).run(case.steps)
    return case, orc


def test_small_case_geometry_bitexact():
    case = W.plain_f64_small()
    print(f"[gpu] geometry {case.name}", flush=True)
    sim = _sim(case, storage="f64")
    _check_geometry(sim, OracleSim(case))
    sim.close()


def test_small_case_fp64_parity(c1_oracle):
    case, orc = c1_oracle
    print(f"[gpu] fp64 parity {case.name} {case.steps} steps", flush=True)
    sim = _sim(case, storage="f64", traj_cap=case.steps)
    sim.step(case.steps)
    sim.status()
    _check_geometry(sim, orc)
    Fo, To, Do = _oracle_traj(orc)
    Fg, Tg, Dg = _gpu_traj(sim, case.steps)
    eF = _rel(Fg, Fo)
    eT = np.abs(Tg - To).max() / (np.abs(Fo).max() * case.bodies[0].radius)
    eD = _rel(Dg[:, :, 0], Do[:, :, 0])
    pg, po = sim.populations(), orc.populations()
    eP = _rel(pg, po)
    ef = np.abs(pg - po).max() / (1.0 / 3.0 + np.abs(po).max())  # on f = w + dF
    print(f"[gpu] errors F {eF:.2e} T {eT:.2e} D {eD:.2e} dF {eP:.2e} f {ef:.2e}", flush=True)
    assert eF < 1e-12 and eT < 1e-12 and eD < 1e-12 and eP < 1e-12
    sim.close()


def test_small_case_fp32_parity(c1_oracle):
    case, orc = c1_oracle
    print(f"[gpu] fp32 parity {case.name}", flush=True)
    sim = _sim(case, storage="f32", traj_cap=case.steps)
    sim.step(case.steps)
    sim.status()
    _check_geometry(sim, orc)
    Fo, To, Do = _oracle_traj(orc)
    Fg, Tg, Dg = _gpu_traj(sim, case.steps)
    eF, eD = _rel(Fg, Fo), _rel(Dg[:, :, 0], Do[:, :, 0])
    eP = _rel(sim.populations(), orc.populations())
    print(f"[gpu] fp32 errors F {eF:.2e} D {eD:.2e} dF {eP:.2e}", flush=True)
    assert eF < 1e-5 and eD < 1e-5 and eP < 1e-5
    sim.close()


def test_forced_motion_remap_parity():
    # a kinematic sphere crossing cells: cover and uncover (refill) every few steps
    case = W.forced_motion(steps=80)
    df0 = W.initial_populations(case, seed=11, amp=1e-4)
    print(f"[gpu] forced motion {case.name} {case.steps} steps", flush=True)
    orc = OracleSim(case, df0=df0)
    sim = _sim(case, storage="f64", traj_cap=case.steps, df0=df0)
    events = 0
    for chunk in range(4):
        before = orc.flags.copy()
        orc.run(case.steps // 4)
        sim.step(case.steps // 4)
        events += int(np.count_nonzero(before != orc.flags))
        _check_geometry(sim, orc)
        eP = _rel(sim.populations(), orc.populations())
        print(f"[gpu] forced motion after {orc.n} steps: dF err {eP:.2e}", flush=True)
        assert eP < 1e-12, eP
    Fo, To, Do = _oracle_traj(orc)
    Fg, Tg, Dg = _gpu_traj(sim, case.steps)
    eF = _rel(Fg, Fo)
    print(f"[gpu] forced motion: flag changes {events}, F err {eF:.2e}", flush=True)
    assert events > 50 and eF < 1e-12
    sim.close()


@pytest.mark.parametrize("seed", range(6))
def test_random_small_boxes_fp64(seed):
    case = W.random_small(seed)
    df0 = W.initial_populations(case, seed=100 + seed, amp=1e-3)
    print(f"[gpu] random {case.name} bodies {len(case.bodies)} steps {case.steps}", flush=True)
    orc = OracleSim(case, df0=df0).run(case.steps)
    sim = _sim(case, storage="f64", traj_cap=case.steps, df0=df0)
    sim.step(case.steps)
    sim.status()
    _check_geometry(sim, orc)
    eP = _rel(sim.populations(), orc.populations())
    Fo, To, Do = _oracle_traj(orc)
    Fg, Tg, Dg = _gpu_traj(sim, case.steps)
    eF = _rel(Fg, Fo)
    eT = np.abs(Tg - To).max() / max(np.abs(To).max(), 1e-300)
    print(f"[gpu] random errors dF {eP:.2e} F {eF:.2e} T {eT:.2e}", flush=True)
    assert eP < 1e-12 and eF < 1e-12 and eT < 1e-11
    sim.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "bf16s"])
def test_rest_state_stays_exactly_zero(storage):
    case = W.plain_f64_small()
    case.drives = []
    print(f"[gpu] rest state {storage}", flush=True)
    sim = _sim(case, storage=storage, shift_log2=16)
    sim.step(10)
    F, T = sim.forces()
    assert not np.any(sim.populations()) and not np.any(F) and not np.any(T)
    sim.close()


def test_nonfinite_state_is_reported():
    from paper_1108_0786_amd._abi import LBM_E_UNSTABLE, LbmError
    case = W.plain_f64_small()
    df0 = np.zeros((19, case.nz, case.ny, case.nx))
    df0[:, 16, 16, 20] = np.nan  # a fluid cell next to the middle sphere
    print("[gpu] non-finite state", flush=True)
    sim = _sim(case, storage="f64", df0=df0)
    sim.step(3)
    with pytest.raises(LbmError) as e:
        sim.status()
    assert e.value.code == LBM_E_UNSTABLE
    sim.close()


def test_overlapping_bodies_rejected():
    from paper_1108_0786_amd._abi import LBM_E_OVERLAP, LbmError
    case = W.plain_f64_small()
    case.bodies[1].anchor = (20.0, 16.0, 16.0)  # 4 lu from the middle sphere, r = 3
    with pytest.raises(LbmError) as e:
        _sim(case, storage="f64")
    assert e.value.code == LBM_E_OVERLAP


@pytest.mark.parametrize("tune", [{"graph_steps": 0}, {"graph_steps": 7}, {"block": 128, "xcd_order": 0},
                                  {"xcd_order": 1}, {"block": 512}, {"full_remap": 1}, {"nontemporal": 1},
                                  {"coop_remap": 0}, {"coop_remap": 2}])
def test_launch_options_are_bitwise_identical(tune):
    # graphs, tile sizes, tile order, the remap skip and the mapping by one or
    # by all of a box's workgroups change nothing: the reductions are in fixed
    # order, the skip only omits no-op remaps, and the shared mapping numbers
    # the links in the same cell order.  coop_remap 2 takes the fallback of
    # the shared mapping: the workgroups join, and the first maps alone
    case = W.forced_motion(steps=60)
    print(f"[gpu] launch options {tune}", flush=True)
    ref = _sim(case, storage="f64", traj_cap=60)
    ref.step(60)
    other = _sim(case, storage="f64", traj_cap=60, tune=tune)
    other.step(60)
    assert np.array_equal(ref.populations(), other.populations())
    assert np.array_equal(ref.trajectory(), other.trajectory())
    assert np.array_equal(ref.flags(), other.flags())
    ref.close()
    other.close()


@pytest.mark.parametrize("tune", [{"xcd_order": 1}, {"xcd_order": 1, "block": 128}, {"xcd_order": 1, "block": 512}])
def test_tile_order_on_a_ragged_grid(tune):
    # 45x31x32 cells: 175 tiles of 256 (349 of 128), not a multiple of the 8
    # XCDs, and a partial last tile; the XCD-aware order must still sweep
    # every tile exactly once
    b, s, d = W.swimmer((22.0, 15.0, 16.0), r=3.0, l0=(10.0, 10.0), k=0.05, gamma=0.01,
                        amplitude=2e-4, period=200.0, phase_lag=math.pi / 2)
    case = W.Case("ragged_45x31x32", 45, 31, 32, 1.0, bodies=b, springs=s, drives=[d], steps=60)
    df0 = W.initial_populations(case, seed=11, amp=1e-4)
    print(f"[gpu] ragged grid {tune}", flush=True)
    orc = OracleSim(case, df0=df0).run(60)
    ref = _sim(case, storage="f64", traj_cap=60, df0=df0)
    ref.step(60)
    other = _sim(case, storage="f64", traj_cap=60, df0=df0, tune=tune)
    other.step(60)
    err = np.abs(ref.populations() - orc.populations()).max() / np.abs(orc.populations()).max()
    assert err < 1e-12
    assert np.array_equal(ref.populations(), other.populations())
    assert np.array_equal(ref.trajectory(), other.trajectory())
    assert np.array_equal(ref.flags(), other.flags())
    ref.close()
    other.close()


def _averaged_case(steps=300):
    # tau 0.6: the plain explicit coupling lets a period-2 mode grow here
    b, s, d = W.swimmer((16.0, 12.0, 12.0), r=3.0, l0=(10.0, 10.0), k=0.05, gamma=0.01,
                        amplitude=5e-4, period=400.0, phase_lag=math.pi / 2)
    return W.Case("averaged_32x24x24", 32, 24, 24, 0.6, bodies=b, springs=s, drives=[d], steps=steps,
                  force_average=True)


def test_force_average_fp64_parity():
    case = _averaged_case()
    df0 = W.initial_populations(case, seed=21, amp=1e-4)
    print(f"[gpu] force average {case.name} {case.steps} steps", flush=True)
    orc = OracleSim(case, df0=df0).run(case.steps)
    sim = _sim(case, storage="f64", traj_cap=case.steps, df0=df0)
    sim.step(case.steps)
    sim.status()
    _check_geometry(sim, orc)
    Fo, To, Do = _oracle_traj(orc)
    Fg, Tg, Dg = _gpu_traj(sim, case.steps)
    eF, eD = _rel(Fg, Fo), _rel(Dg[:, :, 0], Do[:, :, 0])
    eP = _rel(sim.populations(), orc.populations())
    print(f"[gpu] force average errors F {eF:.2e} D {eD:.2e} dF {eP:.2e}", flush=True)
    assert eF < 1e-12 and eD < 1e-12 and eP < 1e-12
    sim.close()


def test_capsule_clearance_uses_the_exact_shape():
    # capsules r = 4, cylinder 8, 16 cells apart: side by side (axes along y)
    # they leave 8 cells of fluid; end to end (axes along x) they touch
    from paper_1108_0786_amd._abi import LBM_E_OVERLAP, LbmError
    c45 = math.sqrt(0.5)

    def pair(quat, y=24.0):
        bodies = [W.make_body(W.CAPSULE, 4.0, 400.0, (24.0 + 16.0 * n, y, 24.0), 4.0, quat=quat) for n in range(2)]
        return W.Case("pair", 64, 48, 48, 0.8, bodies=bodies, steps=1)

    print("[gpu] capsule clearance", flush=True)
    _sim(pair((c45, 0.0, 0.0, c45)), storage="f32").close()
    with pytest.raises(LbmError) as e:
        _sim(pair((1.0, 0.0, 0.0, 0.0)), storage="f32")
    assert e.value.code == LBM_E_OVERLAP
    # across the channel the capsule reaches y +- 8: one cell from the wall at 9, not at 8.5
    _sim(pair((c45, 0.0, 0.0, c45), y=9.0), storage="f32").close()
    with pytest.raises(LbmError) as e:
        _sim(pair((c45, 0.0, 0.0, c45), y=8.5), storage="f32")
    assert e.value.code == LBM_E_OVERLAP


def _sixteen_bodies():
    # the library's maximum of 16 bodies: four rows of four spheres along x,
    # springs between neighbours in each row, one drive per row; the rows'
    # bodies are free, prescribed or rotation-locked in turn
    bodies, springs, drives = [], [], []
    for row, (y, z) in enumerate(((12.0, 12.0), (28.0, 12.0), (12.0, 28.0), (28.0, 28.0))):
        base = len(bodies)
        for n in range(4):
            b = W.make_body(W.SPHERE, 3.0, W.bead_mass(3.0), (10.0 + 16.0 * n, y, z))
            b.kinematic = (row + n) % 3 if n else 0
            if b.kinematic == 1:
                b.vel = (0.002, 0.0, 0.0)
            bodies.append(b)
        springs += [W.Spring(base + n + 1, base + n, 0.05, 0.01, 16.0) for n in range(3)]
        drives.append(W.Drive(left=base, middle=base + 1, right=base + 2, amplitude=2e-4, period=100.0 + 20 * row,
                              phase_lag=math.pi / 2))
    return W.Case("sixteen_64x40x40", 64, 40, 40, 1.0, bodies=bodies, springs=springs, drives=drives, steps=60)


def test_sixteen_bodies_fp64_parity():
    case = _sixteen_bodies()
    df0 = W.initial_populations(case, seed=31, amp=1e-4)
    print(f"[gpu] {case.name}: {len(case.bodies)} bodies, {len(case.springs)} springs, {len(case.drives)} drives",
          flush=True)
    orc = OracleSim(case, df0=df0).run(case.steps)
    sim = _sim(case, storage="f64", traj_cap=case.steps, df0=df0)
    sim.step(case.steps)
    sim.status()
    _check_geometry(sim, orc)
    Fo, To, Do = _oracle_traj(orc)
    Fg, Tg, Dg = _gpu_traj(sim, case.steps)
    eF, eD = _rel(Fg, Fo), _rel(Dg, Do)
    eP = _rel(sim.populations(), orc.populations())
    print(f"[gpu] sixteen bodies: F {eF:.2e} D {eD:.2e} dF {eP:.2e}", flush=True)
    assert eF < 1e-12 and eD < 1e-12 and eP < 1e-12
    sim.close()
