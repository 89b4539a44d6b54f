"""Precision form: the capsule swimmers on the 128x64x64 crop, 1000 steps,
with FP64, FP32, shifted-FP16 and shifted-BF16 population storage, against
the FP64 oracle's trajectory (stored by tests/golden/make_goldens.py, which
calls only the oracle).  The error of each storage type is printed; FP64 and
FP32 are held to the parity bars, the 16-bit formats to the bound their
rounding allows, populations included."""
import os

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
# bound on the normalised errors of forces, displacement and centroid velocity
BOUND = {"f64": 1e-12, "f32": 1e-5, "f16s": 3e-2, "bf16s": 3e-1}


@pytest.mark.parametrize("design", ["SCS", "CCC"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "bf16s"])
def test_capsule_crop_against_oracle(design, storage):
    from paper_1108_0786_amd.sim import Sim
    path = os.path.join(GOLD, f"capsule_crop_{design}.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle trajectory missing (run tests/golden/make_goldens.py)")
    gold = np.load(path)
    case = W.capsule_crop(design, storage)
    steps = int(gold["steps"])
    print(f"[gpu] precision {case.name} {storage} {steps} steps", flush=True)
    sim = Sim(case, storage=storage, traj_cap=steps)
    sim.step(steps)
    sim.status()
    tr = sim.trajectory()[:steps]
    F, D = tr[:, :, 9:12], tr[:, :, 0:3]
    eF = np.abs(F - gold["F"]).max() / np.abs(gold["F"]).max()
    eD = np.abs(D[:, :, 0] - gold["D"][:, :, 0]).max() / np.abs(gold["D"][:, :, 0]).max()
    cg = D[:, :, 0].mean(axis=1)
    co = gold["D"][:, :, 0].mean(axis=1)
    # the centroid is the mean of bodies moving in antiphase, much smaller than
    # their displacements: its error is measured on the bodies' scale
    dscale = np.abs(gold["D"][:, :, 0]).max()
    eC = np.abs(cg - co).max() / dscale
    # centroid velocity (per-step displacement of the centroid)
    vg, vo = np.diff(cg), np.diff(co)
    eV = np.abs(vg - vo).max() / np.abs(vo).max()
    df = sim.populations_at(gold["cells"])
    eP = np.abs(df - gold["df"]).max() / np.abs(gold["df"]).max()
    print(f"[gpu] precision {design} {storage}: force {eF:.2e} body displacement {eD:.2e} "
          f"centroid (on the bodies' scale) {eC:.2e} centroid velocity {eV:.2e} populations {eP:.2e}", flush=True)
    assert np.array_equal(sim.flags()[gold["cells"]] & 0x7F, gold["flags"])
    b = BOUND[storage]
    assert eF < b and eD < b and eC < b
    if storage == "f32":
        # the FP32 parity bar holds for the centroid velocity and the
        # populations themselves
        assert eV < b and eP < b
    else:
        # the velocity is the difference of consecutive centroid positions,
        # so its error carries the factor max|D| / max|v| (about 1e3 here)
        # over the displacement error: in FP64 this cancellation alone
        # reaches 1e-12, and the 16-bit formats store coarser populations
        assert eV < 2.0 * b * max(1.0, dscale / np.abs(vo).max())
        assert eP < b
    sim.close()


def _rne_expected(t, storage):
    """float32 values t rounded to the 16-bit format, round to nearest even
    (IEEE 754), back in float32."""
    if storage == "f16s":
        return t.astype(np.float16).astype(np.float32)
    bits = t.view(np.uint32).astype(np.uint64)
    r = ((bits + 0x7FFF + ((bits >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


@pytest.mark.parametrize("storage", ["f16s", "bf16s"])
def test_storage_rounds_to_nearest_even(storage):
    # a box without bodies: importing populations stores them in the 16-bit
    # format (scaled by 2^16) and exporting reads them back, so the export
    # shows the rounding; half the values sit exactly halfway between two
    # representable numbers, where the tie must go to the even one
    from paper_1108_0786_amd.sim import Sim
    case = W.Case("round_trip", 16, 8, 8, 0.8)
    n = 19 * case.ncells
    rng = np.random.default_rng(5)
    if storage == "bf16s":
        hi = rng.integers(0x3A00, 0x3F00, n).astype(np.uint32) << 16       # bf16 numbers, about 5e-4 .. 0.5
        low = np.where(np.arange(n) % 2 == 0, 0x8000, rng.integers(1, 0x10000, n)).astype(np.uint32)
    else:
        exp = rng.integers(117, 133, n).astype(np.uint32)                  # 2^-10 .. 2^5: normal in FP16
        hi = (exp << 23) | (rng.integers(0, 1024, n).astype(np.uint32) << 13)   # FP16-representable
        low = np.where(np.arange(n) % 2 == 0, 0x1000, rng.integers(1, 0x2000, n)).astype(np.uint32)
    t = (hi | low).view(np.float32)
    sign = np.where(rng.random(n) < 0.5, -1.0, 1.0).astype(np.float32)
    t = t * sign
    df = (t.astype(np.float64) * 2.0 ** -16).reshape(19, case.nz, case.ny, case.nx)
    print(f"[gpu] storage round trip {storage}", flush=True)
    sim = Sim(case, storage=storage, shift_log2=16)
    sim.import_populations(df)
    got = sim.populations()
    want = (_rne_expected(t, storage).astype(np.float64) * 2.0 ** -16).reshape(got.shape)
    sim.close()
    assert np.array_equal(got, want)
