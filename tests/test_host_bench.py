"""Host logic of bench.py, without a GPU: the algorithmic byte count of a
sweep launch, the traffic figure's tie to the sweep sources, and the refusal
of runs on more than one GPU."""
import os
import subprocess
import sys

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("storage,s", [("f64", 8), ("f32", 4), ("f16s", 2), ("bf16s", 2)])
def test_sweep_bytes(storage, s):
    case = W.plain_at_scale(storage)
    # every fluid cell reads and writes its 19 populations; every flag is read
    assert bench.sweep_bytes(case, 1000, storage) == 1000 * 19 * 2 * s + case.ncells
    assert bench.sweep_bytes(case, 0, storage) == case.ncells


def test_traffic_is_tied_to_the_sweep_sources(monkeypatch):
    bytes_ = bench.SWEEP_TRAFFIC["bytes"]
    got = bench.measured_traffic()
    assert got in (bytes_, None)
    monkeypatch.setitem(bench.SWEEP_TRAFFIC, "sha256", "0" * 64)
    assert bench.measured_traffic() is None          # sources changed since the counters were taken


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
