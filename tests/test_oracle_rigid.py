"""Pins of the oracle's rigid-body side (Sec. 2.2, Sec. 3, Sec. 4): driving
protocol, spring-damper forces and time integration, checked in vacuum (no
fluid) against the closed-form solution of the linear recurrence, against
the continuous equations of motion of Sec. 4, and against the normal modes
behind the resonances reported there."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import workloads as W
from oracle import rigid, vacuum


def _vacuum(case, steps):
    return vacuum.run(case, steps)


def _linear_system(m, k, g):
    return vacuum.linear_system(m, k, g)


def test_vacuum_matches_exact_discrete_solution():
    # closed form of s_{n+1} = M s_n + Re(c e^{i w n}):
    #   s_n = Re(s_hat e^{i w n}) + M^n (s_0 - Re(s_hat)),  s_hat = (e^{i w} I - M)^{-1} c
    case = W.plain_f64_small()
    m, k, g = case.bodies[0].mass, 0.05, 0.01
    d = case.drives[0]
    a, w, psi = d.amplitude, 2 * math.pi / d.period, d.phase_lag
    steps = 1500
    hist = _vacuum(case, steps)
    M = _linear_system(m, k, g)
    # driving as complex amplitudes: -a sin(wn) = Re(i a e^{iwn}); a sin(wn - psi) = Re(-i a e^{-i psi} e^{iwn})
    Fl = 1j * a
    Fr = -1j * a * np.exp(-1j * psi)
    Fm = -(Fl + Fr)
    Fc = np.array([Fm, Fl, Fr]) / m
    c = np.concatenate([Fc, Fc])
    s_hat = np.linalg.solve(np.exp(1j * w) * np.eye(6) - M, c)
    # M has a Jordan block at 1 (free translation), so M^n is taken by
    # repeated squaring rather than by eigendecomposition
    s0 = np.zeros(6) - np.real(s_hat)
    for n in (1, 10, 333, 1000, 1500):
        hom = np.linalg.matrix_power(M, n) @ s0
        s = np.real(s_hat * np.exp(1j * w * n)) + hom
        got = np.concatenate([hist[n - 1, :, 0], hist[n - 1, :, 1]])
        assert np.allclose(got, s, rtol=0, atol=1e-12 * np.abs(s).max())
        # the oracle's own closed form, written independently of the test's
        assert np.allclose(vacuum.exact(m, k, g, a, w, psi, n), s, rtol=0, atol=1e-12 * np.abs(s).max())


def test_vacuum_total_momentum_stays_zero():
    # driving forces sum to zero (Eq. FB1) and springs are internal
    hist = _vacuum(W.plain_f64_small(), 800)
    p = hist[:, :, 1].sum(axis=1)
    assert np.abs(p).max() < 1e-18


def test_vacuum_follows_continuous_equations_of_motion():
    # Sec. 4: m x_i'' = dL/dx_i + F_damp; with omega dt ~ 0.03 the unit-step
    # integrator agrees with the continuous solution to a few per cent of the
    # amplitude (first-order error in dt)
    case = W.plain_f64_small()
    m, k, g = case.bodies[0].mass, 0.05, 0.01
    d = case.drives[0]
    a, w, psi = d.amplitude, 2 * math.pi / d.period, d.phase_lag
    steps = 600
    hist = _vacuum(case, steps)

    def rhs(t, s):
        x, v = s[:3], s[3:]
        f = np.array([-(-a * math.sin(w * t) + a * math.sin(w * t - psi)),
                      -a * math.sin(w * t), a * math.sin(w * t - psi)])
        xm, xl, xr = x
        vm, vl, vr = v
        fl = -k * (xl - xm) - g * (vl - vm)
        fr = -k * (xr - xm) - g * (vr - vm)
        acc = (f + np.array([-(fl + fr), fl, fr])) / m
        return np.concatenate([v, acc])

    sol = solve_ivp(rhs, (0, steps), np.zeros(6), t_eval=np.arange(1, steps + 1), rtol=1e-10,
                    atol=1e-14)
    x_cont = sol.y[:3].T
    x_disc = hist[:, :, 0]
    amp = np.abs(x_cont).max()
    assert np.abs(x_disc - x_cont).max() < 0.05 * amp


def test_normal_modes_give_the_two_resonances():
    # the free three-body chain has w^2 = 0, k/m, 3k/m: resonances of the
    # driven amplitude at w0 = w and w0 = w/sqrt(3) (Sec. 4)
    m, w = 400.0, 2 * math.pi / 28116
    a = 1e-3

    def amp_left(k):
        g = 2 * 0.07 * math.sqrt(m * k)  # damping ratio 0.07 as in Sec. 4
        M = _linear_system(m, k, g)
        Fl, Fr = 1j * a, -1j * a * np.exp(-1j * math.pi / 2)
        Fc = np.array([-(Fl + Fr), Fl, Fr]) / m
        s_hat = np.linalg.solve(np.exp(1j * w) * np.eye(6) - M, np.concatenate([Fc, Fc]))
        return abs(s_hat[1])

    ratios = np.linspace(0.3, 1.6, 600)  # w0 / w
    amps = np.array([amp_left(m * (r * w) ** 2) for r in ratios])
    peaks = [ratios[i] for i in range(1, len(ratios) - 1) if amps[i] > amps[i - 1] and amps[i] > amps[i + 1]]
    assert len(peaks) == 2
    # the other mode's tail and the damping shift the lower peak by a few per cent
    assert abs(peaks[0] - 1 / math.sqrt(3)) < 0.05 and abs(peaks[1] - 1.0) < 0.01


def test_driving_protocol_signs_and_gating():
    # Eqs. FB1-FB3 with the delay reading; the middle force balances the others
    dv = dict(left=1, middle=0, right=2, amplitude=2.0, period=8.0, phase_lag=math.pi / 2,
              gate_lagged=True, off_left=-1, off_right=-1)
    F = rigid.driving_forces([dv], 1, 3)
    assert math.isclose(F[1][0], -2.0 * math.sin(math.pi / 4))
    assert F[2][0] == 0.0  # gated: omega t < psi
    F = rigid.driving_forces([dv], 3, 3)
    assert math.isclose(F[2][0], 2.0 * math.sin(3 * math.pi / 4 - math.pi / 2))
    assert F[0][0] + F[1][0] + F[2][0] == 0.0
    dv.update(gate_lagged=False, off_left=2, off_right=5)
    F = rigid.driving_forces([dv], 3, 3)
    assert F[1][0] == 0.0 and F[2][0] != 0.0 and F[0][0] == -F[2][0]
