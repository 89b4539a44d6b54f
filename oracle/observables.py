"""Post-processing quantities the paper evaluates on its trajectories (Sec. 5).

* Eq. K and Eq. V_GA: Golestanian-Ajdari geometric factor
      K = 3 r1 r2 r3 / (2 (r1 + r2 + r3)^2) [1/l1^2 + 1/l2^2 - 1/(l1 + l2)^2]
  and small-amplitude swimming velocity u_GA = K d1 d2 omega sin(phi1 - phi2).
* Eq. arms: arm length l_i(t) = l_i_bar + d_i cos(omega t + phi_i), fitted by
  linear least squares over a window (the paper uses the last full period).
* Eqs. Re, ReSwimmer, ReBody: Re = u l / nu; u_swim = Delta / T with Delta the
  displacement of the central body over one period.
* Eq. eff: Lighthill efficiency 6 pi eta r_eff u_swim^2 / <sum F_dri . u>.
"""
from __future__ import annotations

import math

import numpy as np


def ga_factor(r1, r2, r3, l1, l2):
    """Geometric factor K of Eq. K."""
    pre = 3.0 * r1 * r2 * r3 / (2.0 * (r1 + r2 + r3) ** 2)
    return pre * (1.0 / l1 ** 2 + 1.0 / l2 ** 2 - 1.0 / (l1 + l2) ** 2)


def ga_velocity(K, d1, d2, omega, dphi):
    """u_GA of Eq. V_GA."""
    return K * d1 * d2 * omega * math.sin(dphi)


def reynolds(u, length, nu):
    """Eq. Re."""
    return u * length / nu


def fit_arm(t, length, omega):
    """Least-squares fit of Eq. arms; returns (l_bar, d, phi) with d >= 0."""
    t = np.asarray(t, dtype=np.float64)
    A = np.stack([np.ones_like(t), np.cos(omega * t), np.sin(omega * t)], axis=1)
    c, *_ = np.linalg.lstsq(A, np.asarray(length, dtype=np.float64), rcond=None)
    # d cos(wt + phi) = d cos(phi) cos(wt) - d sin(phi) sin(wt)
    d = math.hypot(c[1], c[2])
    phi = math.atan2(-c[2], c[1])
    return float(c[0]), d, phi


def lighthill_efficiency(eta, r_eff, u_swim, mean_power):
    """Eq. eff with the period-averaged driving power in the denominator."""
    return 6.0 * math.pi * eta * r_eff * u_swim ** 2 / mean_power
