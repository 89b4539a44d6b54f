"""Swimmers of the Sec. 5.1 design study, run on the GPU at the paper's size
(200x100x100, tau 2/3, five driving periods of 28116 steps, FP32 storage,
two-step force mean): the three-sphere designs (a) and (q) and the
all-capsule designs (f), (k) and (p).  Post-processed with the Eq. arms fit
and the GA formulas (Eqs. K, V_GA; a capsule counts as a sphere of
diameter 12, as in Sec. 5.3.2) and compared with what the paper reports
(Tables tab:spheres, tab:sphere_params, tab:caps_family1-3 and the
appendix parameter tables).

Asserted, because they follow from the physics and the paper's own findings
rather than from details of its code:
  * the run stays smooth (no step-to-step oscillation of the bodies);
  * the mean arm lengths give the printed GA factors K;
  * the simulated swimming velocity agrees with the GA prediction from the
    fitted arm oscillations as well as the paper's does (its printed error
    bound for the design), with 5 points of slack;
  * the smaller spheres swim faster than the larger ones ((a) vs (q), Sec.
    5.3.1) and the long swimmer of perpendicular capsules (k) is the slowest
    of (f), (k), (p).
Reported only: u_swim and the arm amplitudes against the printed values."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import observables as ob

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
SPHERES = ("a", "q")
_results = {}


def _printed(design):
    """Printed u_swim, u_GA error bound, and arm parameters of a design."""
    if design in SPHERES:
        sw = GOLD["spheres"][design]
        return sw["u_swim"], sw["error_pct_below"], GOLD["sphere_params"][design]
    sw = GOLD["capsule_swim"][design]
    return sw["u_swim"], sw["error_pct_below"], GOLD["capsule_params"][design]


def _run(design):
    from paper_1108_0786_amd.sim import Sim
    case = W.paper_design(design, "f32") if design in SPHERES else W.paper_capsule_design(design, "f32")
    T = int(case.drives[0].period)
    n = 5 * T
    print(f"[gpu] paper scale {case.name}: {n} steps FP32", flush=True)
    sim = Sim(case, storage="f32", traj_cap=n)
    for p in range(5):
        sim.step(T)
        sim.status()
        print(f"[gpu] paper scale {design}: period {p + 1} done", flush=True)
    tr = sim.trajectory()
    sim.close()
    steps = tr[:, 0, 15].astype(np.int64)
    order = np.argsort(steps)
    tr = tr[order]
    assert np.array_equal(tr[:, 0, 15].astype(np.int64), np.arange(n))
    X = np.array([b.anchor[0] for b in case.bodies])[None, :] + tr[:, :, 0]
    V = tr[:, :, 3]
    t = np.arange(4 * T, 5 * T)
    om = 2.0 * math.pi / T
    lb1, d1, p1 = ob.fit_arm(t, X[4 * T:5 * T, 0] - X[4 * T:5 * T, 1], om)
    lb2, d2, p2 = ob.fit_arm(t, X[4 * T:5 * T, 2] - X[4 * T:5 * T, 0], om)
    r = case.bodies[0].radius if design in SPHERES else 6.0
    K = ob.ga_factor(r, r, r, lb1, lb2)
    out = dict(u_swim=(X[5 * T - 1, 0] - X[4 * T - 1, 0]) / T, d1=d1, d2=d2, sin_dphi=math.sin(p1 - p2), K=K,
               u_ga=ob.ga_velocity(K, d1, d2, om, p1 - p2),
               alternating=np.abs(V[1:-1] - 0.5 * (V[:-2] + V[2:])).max(), vmax=np.abs(V).max())
    u_print, err, par = _printed(design)
    print(f"[gpu] paper scale ({design}): u_swim {out['u_swim']:.4e} (printed {u_print}e-6), "
          f"d1 {d1:.3f} (printed {par['d1']}), d2 {d2:.3f} (printed {par['d2']}), "
          f"sin dphi {out['sin_dphi']:.3f} (printed {par['sin_dphi']}), K {K:.5f} (printed {par['K']}), "
          f"u_swim/u_GA {out['u_swim'] / out['u_ga']:.3f} (printed error < {err}%), max |V| {out['vmax']:.2e}, "
          f"alternating part {out['alternating']:.1e}", flush=True)
    return out


@pytest.mark.parametrize("design", ["a", "q", "f", "k", "p"])
def test_design_study_swimmer(design):
    res = _results[design] = _run(design)
    _, err, par = _printed(design)
    assert np.isfinite(res["u_swim"])
    # the remap impulses leave a step-to-step part of about 1e-3 of the peak
    # velocity; the period-2 instability this guards against reaches 0.1-1
    assert res["alternating"] < 1e-2 * res["vmax"]
    assert abs(res["K"] - par["K"]) < 0.00006
    assert abs(res["u_swim"] / res["u_ga"] - 1.0) < err / 100.0 + 0.05
    if design == "q" and "a" in _results:
        assert _results["a"]["u_swim"] > 2.0 * res["u_swim"]
    if design == "p" and "f" in _results and "k" in _results:
        assert _results["k"]["u_swim"] < min(_results["f"]["u_swim"], res["u_swim"])
