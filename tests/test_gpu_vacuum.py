"""The swimmer in vacuum (Sec. 4) on the GPU through ``lbm_vacuum_run``: the
rigid-body step of the coupled path with no fluid, for many systems at once.

Parity: trajectories of a spread of the resonance-sweep systems against the
oracle's step-by-step vacuum run, to 1e-12 of the largest displacement.

The run of Fig. positionPlot (design-study springs and driving, switched off
after five periods): the whole trajectory against the oracle, the centroid at
rest throughout, and the time at which the arms are back at their rest
lengths against the caption's t3 of about 179000 steps (read as the arms
staying within 0.1% of their driven amplitude: flat in the figure).

The sweep of Fig. vacuumVal2: 38 systems (damping ratio 0.07, omega_0 / omega
from 0.316 to 1.950) for the paper's 10^6 steps.  Asserted: the final states
equal the closed-form solution of the discrete recurrence from rest
(oracle.vacuum.exact) to 1e-9; the amplitude of sphere 2 (the left body) over
the last period equals the same closed form's; and the amplitude curve has
its two maxima next to omega_0 = omega / sqrt(3) and omega_0 = omega.  Printed:
the departure of the amplitudes from the continuous model of Sec. 4 (the
Lagrangian with spring damping), a first-order effect of the unit time
step."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import vacuum
from oracle.observables import fit_arm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _params(case):
    m = case.bodies[0].mass
    sp, d = case.springs[0], case.drives[0]
    return m, sp.k, sp.gamma, d.amplitude, 2.0 * math.pi / d.period, d.phase_lag


def test_vacuum_parity_with_oracle():
    from paper_1108_0786_amd.sim import vacuum_run
    cases = W.vacuum_sweep()[::7]
    steps = 3000
    print(f"[gpu] vacuum parity: {len(cases)} systems, {steps} steps", flush=True)
    _, traj = vacuum_run(cases, steps, traj_cap=steps)
    for s, case in enumerate(cases):
        ref = vacuum.run(case, steps)                        # (steps, bodies, [D, V])
        tr = traj[s][np.argsort(traj[s][:, 0, 15])]
        assert np.array_equal(tr[:, 0, 15], np.arange(steps))
        got = np.stack([tr[:, :, 0], tr[:, :, 3]], axis=2)
        err = np.abs(got - ref).max() / np.abs(ref[:, :, 0]).max()
        print(f"[gpu] {case.name}: max error {err:.1e}", flush=True)
        assert err < 1e-12


def _continuous_amplitude(m, k, g, a, w, psi):
    """Steady amplitude of the left body under the continuous equations of
    motion of Sec. 4: (K - w^2 m + i w G) X = F for the three-body chain."""
    K = np.array([[-2 * k, k, k], [k, -k, 0.0], [k, 0.0, -k]])
    G = np.array([[-2 * g, g, g], [g, -g, 0.0], [g, 0.0, -g]])
    Fl, Fr = 1j * a, -1j * a * np.exp(-1j * psi)
    F = np.array([-(Fl + Fr), Fl, Fr])
    X = np.linalg.solve(-K - w * w * m * np.eye(3) - 1j * w * G, F)
    return abs(X[1])


def test_vacuum_resonance_sweep():
    from paper_1108_0786_amd.sim import vacuum_run
    cases = W.vacuum_sweep()
    steps = cases[0].steps
    T = int(cases[0].drives[0].period)
    print(f"[gpu] vacuum sweep: {len(cases)} systems, {steps} steps", flush=True)
    torch.cuda.synchronize()
    states, traj = vacuum_run(cases, steps, traj_cap=T)
    ratios, amp, amp_exact, amp_cont = [], [], [], []
    worst = 0.0
    for s, case in enumerate(cases):
        m, k, g, a, w, psi = _params(case)
        # final state against the closed form from rest
        exact = vacuum.exact(m, k, g, a, w, psi, steps)
        got = np.array([b["D"][0] for b in states[s]] + [b["V"][0] for b in states[s]])
        err = np.abs(got - exact).max() / np.abs(exact[:3]).max()
        worst = max(worst, err)
        assert err < 1e-9, (case.name, err)
        # amplitude of sphere 2 (the left body) over the last period, and the
        # closed form's over the same steps
        tr = traj[s][np.argsort(traj[s][:, 0, 15])]
        n = tr[:, 0, 15].astype(np.int64)
        assert np.array_equal(n, np.arange(steps - T, steps))
        x = tr[:, 1, 0]
        M = vacuum.linear_system(m, k, g)
        s_hat = vacuum.steady_response(m, k, g, a, w, psi)
        hom = np.linalg.matrix_power(M, steps - T + 1) @ np.real(s_hat)
        xs = np.empty(T)
        for i in range(T):                        # s_{n+1} after step n
            xs[i] = np.real(s_hat[1] * np.exp(1j * w * (steps - T + 1 + i))) - hom[1]
            hom = M @ hom
        A = fit_arm(n, x, w)[1]
        A_exact = fit_arm(n, xs, w)[1]
        assert abs(A - A_exact) < 1e-9 * A_exact
        ratios.append(math.sqrt(k / m) / w)
        amp.append(A / a)
        amp_exact.append(abs(s_hat[1]) / a)
        amp_cont.append(_continuous_amplitude(m, k, g, a, w, psi) / a)
    ratios, amp = np.array(ratios), np.array(amp)
    dev = np.abs(np.array(amp_exact) / np.array(amp_cont) - 1.0)
    print(f"[gpu] vacuum sweep: final states within {worst:.1e} of the closed form; "
          f"steady amplitude / continuous model - 1: {dev.min():.1e} .. {dev.max():.1e}", flush=True)
    for r, A in zip(ratios, amp):
        print(f"[gpu]   w0/w {r:.4f}  A/a {A:.6e}", flush=True)
    peaks = [i for i in range(1, len(amp) - 1) if amp[i] > amp[i - 1] and amp[i] > amp[i + 1]]
    step = ratios[1] - ratios[0]
    assert len(peaks) == 2
    assert abs(ratios[peaks[0]] - 1.0 / math.sqrt(3.0)) < 1.5 * step
    assert abs(ratios[peaks[1]] - 1.0) < 1.5 * step


def test_position_plot_run():
    from paper_1108_0786_amd.sim import vacuum_run
    case = W.vacuum_position_plot()
    n = case.steps
    T = int(case.drives[0].period)
    print(f"[gpu] vacuum run of Fig. positionPlot: {n} steps", flush=True)
    _, traj = vacuum_run([case], n, traj_cap=n)
    tr = traj[0][np.argsort(traj[0][:, 0, 15])]
    assert np.array_equal(tr[:, 0, 15], np.arange(n))
    ref = vacuum.run(case, n)
    D = tr[:, :, 0]
    err = np.abs(D - ref[:, :, 0]).max() / np.abs(ref[:, :, 0]).max()
    # force neutrality: the driving forces and the springs sum to zero
    drift = np.abs(D.mean(axis=1)).max()
    arms = np.maximum(np.abs(D[:, 0] - D[:, 1]), np.abs(D[:, 2] - D[:, 0]))
    amp = arms[4 * T:5 * T].max()
    t3 = int(np.where(arms > 1e-3 * amp)[0][-1]) + 1
    print(f"[gpu] positionPlot: error against the oracle {err:.1e}, centroid drift {drift:.1e}, driven arm "
          f"amplitude {amp:.3f} cells, arms at rest (0.1%) from step {t3} (caption: about 179000)", flush=True)
    assert err < 1e-12
    assert drift < 1e-9 * amp
    assert abs(t3 - 179000) < 0.05 * 179000
