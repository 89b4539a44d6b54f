"""Object mapping, flag changes, boundary links and momentum exchange (Sec. 2.3).

Readings of points the paper leaves open:

* "Cell centre inside an object": the centre of cell (i, j, k) is
  (i+1/2, j+1/2, k+1/2); it is inside a sphere when its squared distance from
  the centre is <= r^2 (closed ball) and inside a capsule when its squared
  distance from the capsule's axis segment is <= r^2.  Periodic axes use the
  minimum image.
* The geometry is evaluated in a fixed sequence of float64 operations so that
  any other implementation that follows the same sequence reaches the same
  inside/outside decision bit for bit:
    R = floor(X) componentwise, f = X - R;
    d = cell index - R (integer; on periodic axes wrapped into [-L//2, L - L//2));
    r = (d + 0.5) - f;
    sphere:  (r_x r_x + r_y r_y) + r_z r_z <= radius * radius;
    capsule: axis a = local x of the quaternion q = (w, x, y, z):
               a = (1 - 2 (q_y q_y + q_z q_z), 2 (q_x q_y + q_w q_z), 2 (q_x q_z - q_w q_y)),
             t = clamp((r_x a_x + r_y a_y) + r_z a_z, -h, h), s = r - t a,
             (s_x s_x + s_y s_y) + s_z s_z <= radius * radius;
    slab (test only, the moving wall of a Couette cell): r.a > 0.
  No fused multiply-add is implied.
* The same offset r is the lever arm of the torque and the point at which the
  object's velocity u_w = V + Omega x r is evaluated (rotation included, Sec. 2.3).
* Refill of uncovered cells: the missing populations are set to the
  equilibrium at the previous owner's velocity at the cell's centre, with the
  density averaged over the D3Q19 neighbours that are fluid both before and
  after the remap (rho = 1 when there is none).  Covered cells simply stop
  being fluid; their populations are discarded (the paper does not say where
  their mass and momentum go).
* Eq. hydroF sums alpha from 1 to 19 while the directions are numbered 0..18;
  the rest direction carries no momentum, so the sum is over the 18 moving
  directions.  The torque, which the paper implies (u_w includes rotation) but
  does not print, is the sum of r x (link term) with r the lever arm above.
* Deviation form of Eq. hydroF: 2 f~ = 2 dF~ + 2 w, so the force splits into
  a part from the deviations and the geometric part sum 2 w_alpha e_alpha,
  which depends only on the link set.  The geometric part is accumulated in
  integers (36 * 2 w_alpha is 4 or 2), so it is exact, and is exactly zero for
  a body with mirror-symmetric link set.
"""
from __future__ import annotations

import math

import numpy as np

from .d3q19 import E, W, OPP, Q, TWO_W_36

SPHERE, CAPSULE, SLAB = 0, 1, 2


def real(x):
    return np.real(x)


def quat_axis(q):
    """Local x axis of the rotation q = (w, x, y, z)."""
    qw, qx, qy, qz = q
    ax = 1.0 - 2.0 * (qy * qy + qz * qz)
    ay = 2.0 * (qx * qy + qw * qz)
    az = 2.0 * (qx * qz - qw * qy)
    return ax, ay, az


def lever_arms(X, cells, dims, periodic):
    """r = (d + 1/2) - f for the given flat cell indices, relative to position X
    (float64 or complex128 3-vector), following the fixed operation sequence of
    the module docstring.  Returns three arrays."""
    nx, ny, nz = dims
    i = cells % nx
    j = (cells // nx) % ny
    k = cells // (nx * ny)
    idx = (i, j, k)
    out = []
    for d in range(3):
        R = math.floor(float(real(X[d])))
        f = X[d] - R
        di = idx[d] - R
        if periodic[d]:
            L = dims[d]
            di = (di + L // 2) % L - L // 2
        out.append((di + 0.5) - f)
    return out


def inside(body, r):
    """Inside test of Sec. 2.3 (module docstring) on lever arms r (real parts)."""
    rx, ry, rz = (real(v) for v in r)
    rad2 = body["radius"] * body["radius"]
    if body["shape"] == SPHERE:
        return (rx * rx + ry * ry) + rz * rz <= rad2
    ax, ay, az = (float(real(v)) for v in quat_axis(body["quat"]))
    t = (rx * ax + ry * ay) + rz * az
    if body["shape"] == SLAB:
        return t > 0.0
    h = body["half_len"]
    t = np.minimum(np.maximum(t, -h), h)
    sx = rx - t * ax
    sy = ry - t * ay
    sz = rz - t * az
    return (sx * sx + sy * sy) + sz * sz <= rad2


def map_bodies(bodies, dims, periodic):
    """Flag field of Alg. 2 (map S to lattice grid): 0 = fluid, 1 + b = object b.
    A cell inside several objects (not allowed by the input checks) takes the
    lowest index."""
    nx, ny, nz = dims
    n = nx * ny * nz
    flags = np.zeros(n, dtype=np.uint8)
    cells = np.arange(n, dtype=np.int64)
    for b in reversed(range(len(bodies))):
        body = bodies[b]
        r = lever_arms(body["X"], cells, dims, periodic)
        flags[inside(body, r)] = 1 + b
    return flags


def wall_velocity(body, cells, dims, periodic):
    """u_w = V + Omega x r at the centres of ``cells`` (Sec. 2.3)."""
    rx, ry, rz = lever_arms(body["X"], cells, dims, periodic)
    V = body["V"]
    O = body["Omega"]
    return (V[0] + (O[1] * rz - O[2] * ry),
            V[1] + (O[2] * rx - O[0] * rz),
            V[2] + (O[0] * ry - O[1] * rx))


def links(flags, nbr):
    """Boundary links {(x_f, alpha, b)}: fluid cell x_f whose neighbour
    x_f + e_alpha lies in object b; sorted by (x_f, alpha)."""
    fluid = np.nonzero(flags == 0)[0]
    cs, ds, bs = [], [], []
    for a in range(1, Q):
        t = nbr[a, fluid]
        ok = t >= 0
        tf = np.zeros_like(t)
        tf[ok] = flags[t[ok]]
        sel = tf > 0
        cs.append(fluid[sel])
        ds.append(np.full(int(sel.sum()), a, dtype=np.int64))
        bs.append(tf[sel].astype(np.int64) - 1)
    c = np.concatenate(cs)
    d = np.concatenate(ds)
    b = np.concatenate(bs)
    order = np.lexsort((d, c))
    return c[order], d[order], b[order]


def refill(df, old_flags, new_flags, nbr, bodies, dims, periodic):
    """Flag changes of Sec. 2.3: cells that leave an object get equilibrium
    populations at the object's local velocity and the mean density of their
    neighbours that are fluid before and after the remap; cells that enter an
    object lose their populations.  ``df`` (19, N) is modified in place and the
    numbers of uncovered and covered cells are returned."""
    uncovered = np.nonzero((old_flags > 0) & (new_flags == 0))[0]
    covered = np.nonzero((old_flags == 0) & (new_flags > 0))[0]
    if uncovered.size:
        for c in uncovered:
            total = 0.0
            count = 0
            for a in range(1, Q):
                n = nbr[a, c]
                if n < 0 or old_flags[n] != 0 or new_flags[n] != 0:
                    continue
                s = df[0, n]
                for q in range(1, Q):
                    s = s + df[q, n]
                total = total + s
                count += 1
            drho = total / count if count else 0.0 * total
            rho = 1.0 + drho
            b = int(old_flags[c]) - 1
            u = wall_velocity(bodies[b], np.array([c]), dims, periodic)
            u = [v[0] for v in u]
            usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
            for a in range(Q):
                eu = E[a, 0] * u[0] + E[a, 1] * u[1] + E[a, 2] * u[2]
                df[a, c] = W[a] * (drho + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq))
    solid = new_flags > 0
    df[:, solid] = 0.0
    return int(uncovered.size), int(covered.size)


def _fsum(x):
    x = np.asarray(x)
    if np.iscomplexobj(x):
        return math.fsum(x.real.tolist()) + 1j * math.fsum(x.imag.tolist())
    return math.fsum(x.tolist())


def momentum_exchange(link_c, link_d, link_b, dft, rho, bodies, dims, periodic, nbr):
    """Hydrodynamic force and torque on every object (Eq. hydroF):

      F_b = sum over links of e_alpha [2 f~_alpha(x_f) + 6 w_alpha rho(x_f) e_opp.u_w(x_f + e_alpha)]

    with f~ = w + dF~.  The deviation part is summed with math.fsum (a
    correctly rounded sum, independent of order); the geometric part
    2 w_alpha e_alpha (and its torque) is summed exactly in integers.
    Returns (F, T) as lists of 3-vectors, one per object."""
    y = nbr[link_d, link_c]
    return link_forces(link_d, link_b, y, dft[link_d, link_c], rho[link_c], bodies, dims, periodic)


def link_forces(link_d, link_b, y, dft_link, rho_link, bodies, dims, periodic):
    """Eq. hydroF from per-link values: direction alpha, body b, body cell y,
    the post-collision deviation dF~_alpha(x_f) and the density rho(x_f)."""
    F_out, T_out = [], []
    for b, body in enumerate(bodies):
        sel = link_b == b
        d = link_d[sel]
        yy = y[sel]
        u = wall_velocity(body, yy, dims, periodic)
        r = lever_arms(body["X"], yy, dims, periodic)
        e = E[d]
        o = OPP[d]
        eu_opp = E[o, 0] * u[0] + E[o, 1] * u[1] + E[o, 2] * u[2]
        s = 2.0 * dft_link[sel] + 6.0 * W[d] * rho_link[sel] * eu_opp
        term = [e[:, 0] * s, e[:, 1] * s, e[:, 2] * s]
        torque = [r[1] * term[2] - r[2] * term[1],
                  r[2] * term[0] - r[0] * term[2],
                  r[0] * term[1] - r[1] * term[0]]
        # geometric part, exact: G = sum e c / 36, S = sum (2 d + 1) x e c, c = 36 * 2 w
        cw = TWO_W_36[d]
        g_int = [int(np.sum(e[:, k] * cw)) for k in range(3)]
        nx, ny, nz = dims
        idx = (yy % nx, (yy // nx) % ny, yy // (nx * ny))
        two_d = []
        fpart = []
        for k in range(3):
            R = math.floor(float(real(body["X"][k])))
            di = idx[k] - R
            if periodic[k]:
                L = dims[k]
                di = (di + L // 2) % L - L // 2
            two_d.append(2 * di + 1)
            fpart.append(body["X"][k] - R)
        ec = [e[:, k] * cw for k in range(3)]
        s_int = [int(np.sum(two_d[1] * ec[2] - two_d[2] * ec[1])),
                 int(np.sum(two_d[2] * ec[0] - two_d[0] * ec[2])),
                 int(np.sum(two_d[0] * ec[1] - two_d[1] * ec[0]))]
        G = [g / 36.0 for g in g_int]
        Tg = [s_int[0] / 72.0 - (fpart[1] * G[2] - fpart[2] * G[1]),
              s_int[1] / 72.0 - (fpart[2] * G[0] - fpart[0] * G[2]),
              s_int[2] / 72.0 - (fpart[0] * G[1] - fpart[1] * G[0])]
        F_out.append([_fsum(term[k]) + G[k] for k in range(3)])
        T_out.append([_fsum(torque[k]) + Tg[k] for k in range(3)])
    return F_out, T_out
