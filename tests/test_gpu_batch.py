"""Batched boxes (one context, one launch per kernel per step for all boxes):
against sequential single-box runs (bitwise identical per box, including
boxes that stop early at their step limit) and against the CPU oracle, box
by box, on boxes of the parameter sweep with different sizes, relaxation
times and coupling forms."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _cases(n, steps):
    cases = W.batched_sweep(seed=7)[:n]
    for c, s in zip(cases, steps):
        c.steps = s
    return cases


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_batched_equals_sequential_bitwise(storage):
    from paper_1108_0786_amd.sim import BatchSim, Sim
    steps = [40, 25, 40, 33]
    cases = _cases(4, steps)
    print(f"[gpu] batch of {len(cases)} ({storage}): " + ", ".join(c.name for c in cases), flush=True)
    batch = BatchSim(cases, storage=storage, traj_cap=max(steps))
    for b, s in enumerate(steps):
        batch.set_step_limit(b, s)
    batch.step(max(steps))
    batch.status()
    for b, c in enumerate(cases):
        assert batch.step_count(b) == steps[b]
        one = Sim(c, storage=storage, traj_cap=max(steps))
        one.step(steps[b])
        assert np.array_equal(one.populations(), batch.populations(b)), c.name
        assert np.array_equal(one.trajectory()[:steps[b]], batch.trajectory(b)[:steps[b]]), c.name
        assert np.array_equal(one.flags(), batch.flags(b))
        one.close()
    batch.close()


def test_autotuner_picks_a_candidate_and_keeps_results(tmp_path, monkeypatch):
    from paper_1108_0786_amd import autotune
    from paper_1108_0786_amd.sim import BatchSim
    monkeypatch.setenv("LBMSWIM_TUNING_CACHE", str(tmp_path / "t.json"))
    cases = _cases(3, [200, 200, 200])
    ref = BatchSim(cases, storage="f32", traj_cap=8)
    tuned = BatchSim(cases, storage="f32", traj_cap=8)
    best = autotune.tune(tuned, steps=16)
    assert best in autotune.CANDIDATES
    assert (tmp_path / "t.json").exists()
    # both contexts advanced by the same number of steps: identical state
    n = tuned.step_count(0)
    ref.step(n)
    for b in range(3):
        assert np.array_equal(ref.populations(b), tuned.populations(b))
    ref.close()
    tuned.close()


# boxes of the seed-7 sweep: two at tau < 0.65 (two-step force mean), three
# at tau = 0.73, 0.93 and 1.19 (plain coupling of Alg. 2), three box shapes
ORACLE_BOXES = (6, 37, 50, 9, 65)


@pytest.fixture(scope="module")
def sweep_oracle():
    from oracle_jobs import run_many
    cases = W.batched_sweep(seed=7)
    picked = [cases[i] for i in ORACLE_BOXES]
    steps = [150, 150, 150, 150, 120]
    print("[gpu] oracle runs of " + ", ".join(f"{c.name} (tau {c.tau:.3f}, force mean {c.force_average})"
                                            for c in picked), flush=True)
    return picked, steps, run_many(list(zip(picked, steps)), workers=5)


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_batched_boxes_against_oracle(sweep_oracle, storage, tol):
    from paper_1108_0786_amd.sim import BatchSim
    cases, steps, gold = sweep_oracle
    assert any(c.force_average for c in cases) and any(not c.force_average for c in cases)
    print(f"[gpu] batch of {len(cases)} against the oracle ({storage})", flush=True)
    batch = BatchSim(cases, storage=storage, traj_cap=max(steps))
    for b, s in enumerate(steps):
        batch.set_step_limit(b, s)
    batch.step(max(steps))
    batch.status()
    for b, (c, s, (F, T, D, V, df, flags)) in enumerate(zip(cases, steps, gold)):
        assert batch.step_count(b) == s
        tr = batch.trajectory(b)[:s]
        eF = np.abs(tr[:, :, 9:12] - F).max() / np.abs(F).max()
        eD = np.abs(tr[:, :, 0] - D[:, :, 0]).max() / np.abs(D[:, :, 0]).max()
        eV = np.abs(tr[:, :, 3] - V[:, :, 0]).max() / np.abs(V[:, :, 0]).max()
        pg = batch.populations(b)
        eP = np.abs(pg - df).max() / np.abs(df).max()
        print(f"[gpu] {c.name} {storage}: F {eF:.2e} D {eD:.2e} V {eV:.2e} dF {eP:.2e}", flush=True)
        assert np.array_equal(batch.flags(b) & 0x7F, flags), c.name
        assert eF < tol and eD < tol and eV < tol and eP < tol, c.name
    batch.close()


@pytest.mark.parametrize("coop", [1, 2])
def test_shared_mapping_in_a_batch_bitwise(coop):
    # eight boxes whose bodies remap, each with its own join words: the shared
    # mapping (1) and its fallback with the workgroups joined (2) give the
    # one-workgroup mapping's results bit for bit
    from paper_1108_0786_amd.sim import BatchSim
    steps = 60
    cases = [W.forced_motion(steps=steps) for _ in range(8)]
    print(f"[gpu] shared mapping in a batch of {len(cases)}, coop {coop}", flush=True)
    out = []
    for c in (0, coop):
        b = BatchSim(cases, storage="f64", traj_cap=steps, tune={"coop_remap": c})
        b.step(steps)
        b.status()
        out.append([(b.populations(i), b.trajectory(i), b.flags(i)) for i in range(len(cases))])
        b.close()
    for (p0, t0, f0), (p1, t1, f1) in zip(*out):
        assert np.array_equal(p0, p1) and np.array_equal(t0, t1) and np.array_equal(f0, f1)
