"""LBGK D3Q19 collision and streaming with bounce-back (Sec. 2.1 and 2.3).

Deviation form.  The oracle stores dF_alpha = f_alpha - w_alpha instead of
f_alpha.  This is an exact change of variables (the rest state f = w becomes
dF = 0) that keeps the small deviations of a slow flow from being rounded
against the O(0.1) rest weights; every formula below is the paper's formula
with f replaced by w + dF.

Readings of points the paper leaves open:

* The equilibrium is not printed (Eq. lbgk only names it); the oracle uses the
  second-order polynomial equilibrium of the cited D3Q19 LBGK model,
  f_eq = w rho (1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u.u), with rho = sum f and
  rho u = sum e f.
* Eq. lbm:bounce_back writes both sides at time t; it is read as halfway link
  bounce-back: the post-collision population that would leave the fluid cell
  through a wall comes back in the opposite direction at t+1 in the same cell.
* In the moving-object rule of Sec. 2.3, rho_w is the pre-collision density of
  the fluid cell (equal to the post-collision one, since LBGK conserves mass)
  and u_w is the object's velocity at the centre of the object cell
  x_f + e_alpha, rotation included.
* Test-only forcing: a uniform body force g (used only to pin the oracle
  against Poiseuille flow and Hasimoto drag) enters through Guo's scheme,
  u = (rho u + g/2)/rho and the source (1 - 1/(2 tau)) w [3(e - u) + 9 (e.u) e].g.
  The method itself has no body force.
"""
from __future__ import annotations

import numpy as np

from .d3q19 import E, W, OPP, Q


def moments(df):
    """Density deviation drho = rho - 1 = sum_alpha dF_alpha and momentum
    j = sum_alpha e_alpha dF_alpha (Sec. 2.1; the rest weights sum to 1 and carry
    no momentum).  ``df`` has shape (19, ...); sums run over alpha = 0..18 in
    order.  The density deviation is kept apart from the 1 so that it is not
    rounded against it."""
    s = df[0].copy()
    for a in range(1, Q):
        s = s + df[a]
    drho = s
    j = []
    for d in range(3):
        acc = np.zeros_like(df[0])
        for a in range(1, Q):
            if E[a, d] == 1:
                acc = acc + df[a]
            elif E[a, d] == -1:
                acc = acc - df[a]
        j.append(acc)
    return drho, j


def equilibrium_dev(drho, u):
    """dF_eq_alpha = f_eq_alpha(rho, u) - w_alpha
    = w_alpha [drho + rho (3 e.u + 4.5 (e.u)^2 - 1.5 u.u)],  rho = 1 + drho  (Eq. lbgk)."""
    usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    rho = 1.0 + drho
    out = []
    for a in range(Q):
        eu = E[a, 0] * u[0] + E[a, 1] * u[1] + E[a, 2] * u[2]
        out.append(W[a] * (drho + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq)))
    return np.stack(out)


def collide(df, tau, g=None):
    """Post-collision deviations (Eq. collide):
    dF~ = dF - (dF - dF_eq(rho, u)) / tau.

    Returns (dF~, rho, u).  With the test-only force ``g`` the velocity and the
    source term follow Guo's scheme (module docstring)."""
    drho, j = moments(df)
    rho = 1.0 + drho
    if g is None:
        u = [j[d] / rho for d in range(3)]
    else:
        u = [(j[d] + 0.5 * g[d]) / rho for d in range(3)]
    dfeq = equilibrium_dev(drho, u)
    dft = df - (df - dfeq) / tau
    if g is not None:
        pref = 1.0 - 0.5 / tau
        for a in range(1, Q):
            eu = E[a, 0] * u[0] + E[a, 1] * u[1] + E[a, 2] * u[2]
            src = 0.0
            for d in range(3):
                src = src + (3.0 * (E[a, d] - u[d]) + 9.0 * eu * E[a, d]) * g[d]
            dft[a] = dft[a] + pref * W[a] * src
        a = 0
        src = 0.0
        for d in range(3):
            src = src + (3.0 * (0.0 - u[d])) * g[d]
        dft[0] = dft[0] + pref * W[0] * src
    return dft, rho, u


def neighbour_table(nx, ny, nz, periodic):
    """nbr[alpha, c] = linear index of cell c + e_alpha, or -1 where that step
    leaves the box through a non-periodic face (a wall)."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    k = k.ravel()
    n = np.array([nx, ny, nz])
    nbr = np.empty((Q, nx * ny * nz), dtype=np.int64)
    for a in range(Q):
        t = [i + E[a, 0], j + E[a, 1], k + E[a, 2]]
        ok = np.ones_like(i, dtype=bool)
        for d in range(3):
            if periodic[d]:
                t[d] = t[d] % n[d]
            else:
                ok &= (t[d] >= 0) & (t[d] < n[d])
        idx = t[0] + nx * (t[1] + ny * t[2])
        nbr[a] = np.where(ok, idx, -1)
    return nbr


def stream_bounce_back(dft, rho, flags, nbr, wall_velocity):
    """Streaming (Eq. streaming) with halfway bounce-back at walls
    (Eq. lbm:bounce_back) and at moving objects (Sec. 2.3), in push form.

    For every fluid cell x and alpha = 1..18, with y = x + e_alpha:
      y fluid          -> dF_alpha(y, t+1)    = dF~_alpha(x)
      y beyond a wall  -> dF_opp(alpha)(x,t+1) = dF~_alpha(x)
      y in object b    -> dF_opp(alpha)(x,t+1) = dF~_alpha(x)
                                                + 6 w_alpha rho(x) e_opp(alpha).u_b(y)
    and dF_0(x, t+1) = dF~_0(x) (f_0 does not stream).  Since w is symmetric
    the rest weights cancel on both sides of every rule, so the rules hold for
    the deviations as written.

    ``dft`` and the result have shape (19, N) (flattened cells); ``flags`` is
    (N,) with 0 = fluid and 1 + b = object b; ``wall_velocity(b, cells)``
    returns the velocity of object b at those cells' centres as three arrays.
    """
    new = np.zeros_like(dft)
    fluid = np.nonzero(flags == 0)[0]
    new[0, fluid] = dft[0, fluid]
    for a in range(1, Q):
        o = OPP[a]
        tgt = nbr[a, fluid]
        wall = tgt < 0
        tflag = np.where(wall, 0, flags[np.where(wall, 0, tgt)])
        to_fluid = (~wall) & (tflag == 0)
        to_body = (~wall) & (tflag > 0)
        new[a, tgt[to_fluid]] = dft[a, fluid[to_fluid]]
        xs = fluid[wall]
        new[o, xs] = dft[a, xs]
        if np.any(to_body):
            xs = fluid[to_body]
            ys = tgt[to_body]
            bs = tflag[to_body].astype(np.int64) - 1
            eu = np.zeros(xs.shape, dtype=dft.dtype)
            for b in np.unique(bs):
                sel = bs == b
                u = wall_velocity(int(b), ys[sel])
                eu[sel] = E[o, 0] * u[0] + E[o, 1] * u[1] + E[o, 2] * u[2]
            new[o, xs] = dft[a, xs] + 6.0 * W[a] * rho[xs] * eu
    return new
