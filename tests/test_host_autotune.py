"""Host logic of the launch-shape autotuner, without a GPU: the cache key,
the JSON cache, the cached path (no timing run) and the choice of the
fastest candidate (on a stand-in context whose step time depends on the
tuning, with the device synchronisation stubbed out)."""
import json
import time
from types import SimpleNamespace

import pytest

from paper_1108_0786_amd import autotune

torch = pytest.importorskip("torch")


class FakeSim:
    """Records lbm_tune calls; a step sleeps unless the tuning is `fast`."""

    def __init__(self, shapes, storage="f32", fast=None):
        self.storage = storage
        self.boxes = [SimpleNamespace(case=SimpleNamespace(nx=a, ny=b, nz=c)) for a, b, c in shapes]
        self.fast = fast or {}
        self.current = {}
        self.calls = []

    def tune(self, key, value):
        self.current[key] = value
        self.calls.append((key, value))

    def step(self, n):
        slow = any(self.current.get(k) != v for k, v in self.fast.items())
        if slow:
            time.sleep(2e-4 * n)


def test_key_lists_each_shape_once_in_order():
    sim = FakeSim([(64, 32, 32), (32, 32, 32), (64, 32, 32)], storage="f16s")
    assert autotune.key_of(sim) == "f16s|3|32x32x32;64x32x32"


def test_cache_round_trip(tmp_path, monkeypatch):
    monkeypatch.setenv("LBMSWIM_TUNING_CACHE", str(tmp_path / "sub" / "tuning.json"))
    assert autotune._load() == {}
    autotune._store({"k": {"tuning": {"block": 512}, "us_per_step": 1.0}})
    assert autotune._load() == {"k": {"tuning": {"block": 512}, "us_per_step": 1.0}}
    (tmp_path / "sub" / "tuning.json").write_text("not json")
    assert autotune._load() == {}


def test_cached_tuning_is_applied_without_a_timing_run(tmp_path, monkeypatch):
    path = tmp_path / "tuning.json"
    monkeypatch.setenv("LBMSWIM_TUNING_CACHE", str(path))
    sim = FakeSim([(48, 32, 32)])
    want = {"block": 128, "xcd_order": 1, "graph_steps": 64}
    path.write_text(json.dumps({autotune.key_of(sim): {"tuning": want, "us_per_step": 3.0}}))

    def no_steps(n):
        raise AssertionError("a cached tuning must not run the simulation")
    sim.step = no_steps
    assert autotune.tune(sim) == want
    assert sim.current == want


def test_fastest_candidate_is_chosen_and_cached(tmp_path, monkeypatch):
    monkeypatch.setenv("LBMSWIM_TUNING_CACHE", str(tmp_path / "tuning.json"))
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    fast = {"block": 512, "xcd_order": 0, "graph_steps": 16}
    assert fast in autotune.CANDIDATES
    sim = FakeSim([(64, 64, 64)], fast=fast)
    best = autotune.tune(sim, steps=8)
    assert best == fast
    assert sim.current == fast                      # the winner is left applied
    table = json.loads((tmp_path / "tuning.json").read_text())
    assert table[autotune.key_of(sim)]["tuning"] == fast
    # every candidate was tried once
    tried = {tuple(sorted(c.items())) for c in autotune.CANDIDATES}
    assert len(tried) == len(autotune.CANDIDATES)
    assert sum(1 for k, _ in sim.calls if k == "block") == len(autotune.CANDIDATES) + 1


class RecordingSim(FakeSim):
    """Records the graph length in force at every step call."""

    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        self.runs = []

    def step(self, n):
        self.runs.append((self.current.get("graph_steps"), n))


def test_timed_steps_cover_whole_graphs():
    assert autotune.timed_steps(32, 64) == 64
    assert autotune.timed_steps(32, 16) == 32
    assert autotune.timed_steps(40, 16) == 48
    assert autotune.timed_steps(5, 0) == 5


def test_graph_candidates_are_timed_with_their_graphs(tmp_path, monkeypatch):
    # every timing run of a candidate is a whole, non-zero number of its
    # graphs, so that lbm_step replays the captured graph it would use
    monkeypatch.setenv("LBMSWIM_TUNING_CACHE", str(tmp_path / "tuning.json"))
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    sim = RecordingSim([(96, 48, 48)])
    autotune.tune(sim, steps=32)
    timed = sim.runs[1::2]          # each candidate: warm-up run, then timed run
    assert len(timed) == len(autotune.CANDIDATES)
    for g, n in timed:
        assert g > 0 and n >= g and n % g == 0, (g, n)
