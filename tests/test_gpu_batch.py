"""Batched boxes (one context, one launch per kernel per step for all boxes)
against sequential single-box runs: bitwise identical per box, including
boxes that stop early at their step limit."""
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
