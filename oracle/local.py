"""One coupled step evaluated at chosen cells only (Sec. 2.1 and 2.3).

For boxes too large to hold whole in the oracle, the results of a GPU step
are checked cell by cell: given the pre-collision deviations dF^n at the
target cells and their D3Q19 neighbours, the flags of step n and the body
states of step n, these functions give dF^{n+1} at the targets and the
momentum-exchange force and torque of every body.  They restate the rules
of ``oracle.lbm.stream_bounce_back`` in pull form (what arrives at a target
cell y in direction alpha came from y - e_alpha):

  source fluid         -> dF^{n+1}_alpha(y) = dF~_alpha(y - e_alpha)
  source beyond a wall -> dF^{n+1}_alpha(y) = dF~_opp(alpha)(y)
  source in body b     -> dF^{n+1}_alpha(y) = dF~_opp(alpha)(y)
                                              + 6 w_alpha rho(y) e_alpha.u_b(y - e_alpha)
and dF^{n+1}_0(y) = dF~_0(y).
"""
from __future__ import annotations

import numpy as np

from . import coupling, lbm
from .d3q19 import E, OPP, Q, W


def neighbours(cells, dims, periodic, sign=1):
    """(19, n) linear indices of cells + sign * e_alpha, -1 beyond a wall."""
    nx, ny, nz = dims
    cells = np.asarray(cells, dtype=np.int64)
    i, j, k = cells % nx, (cells // nx) % ny, cells // (nx * ny)
    out = np.empty((Q, cells.size), dtype=np.int64)
    n = (nx, ny, nz)
    for a in range(Q):
        t = [i + sign * E[a, 0], j + sign * E[a, 1], k + sign * E[a, 2]]
        ok = np.ones(cells.size, dtype=bool)
        for d in range(3):
            if periodic[d]:
                t[d] = t[d] % n[d]
            else:
                ok &= (t[d] >= 0) & (t[d] < n[d])
        out[a] = np.where(ok, t[0] + nx * (t[1] + ny * t[2]), -1)
    return out


class Known:
    """Pre-collision deviations known at a set of cells (19 x n, cells sorted)."""

    def __init__(self, cells, df):
        order = np.argsort(cells)
        self.cells = np.asarray(cells, dtype=np.int64)[order]
        self.df = np.asarray(df)[:, order]

    def index(self, cells):
        pos = np.searchsorted(self.cells, cells)
        pos = np.minimum(pos, self.cells.size - 1)
        if not np.all(self.cells[pos] == cells):
            raise KeyError("a needed cell was not provided")
        return pos


def collide_at(known, cells, tau):
    pos = known.index(cells)
    return lbm.collide(known.df[:, pos], tau)


def step_at(known, targets, flags, bodies, dims, periodic, tau):
    """dF^{n+1} (19, len(targets)) at fluid targets; ``flags`` is the full
    flag field of step n (0 fluid, 1 + b body b)."""
    targets = np.asarray(targets, dtype=np.int64)
    src = neighbours(targets, dims, periodic, sign=-1)     # y - e_alpha
    dft_y, rho_y, _ = collide_at(known, targets, tau)
    out = np.zeros((Q, targets.size))
    out[0] = dft_y[0]
    for a in range(1, Q):
        o = OPP[a]
        x = src[a]
        wall = x < 0
        xf = np.where(wall, 0, x)
        xflag = np.where(wall, 0, flags[xf])
        fluid = (~wall) & (xflag == 0)
        body = (~wall) & (xflag > 0)
        if np.any(fluid):
            dft_x, _, _ = collide_at(known, x[fluid], tau)
            out[a, fluid] = dft_x[a]
        out[a, wall] = dft_y[o, wall]
        if np.any(body):
            for b in np.unique(xflag[body]):
                sel = body & (xflag == b)
                u = coupling.wall_velocity(bodies[int(b) - 1], x[sel], dims, periodic)
                eu = E[a, 0] * u[0] + E[a, 1] * u[1] + E[a, 2] * u[2]
                out[a, sel] = dft_y[o, sel] + 6.0 * W[o] * rho_y[sel] * eu
    return out


def links_at(cells, flags, dims, periodic):
    """Boundary links (cell, alpha, body) of the given fluid cells, sorted."""
    cells = np.asarray(cells, dtype=np.int64)
    cells = cells[flags[cells] == 0]
    nb = neighbours(cells, dims, periodic)
    cs, ds, bs = [], [], []
    for a in range(1, Q):
        t = nb[a]
        ok = t >= 0
        tf = np.zeros(t.size, dtype=np.int64)
        tf[ok] = flags[t[ok]]
        sel = tf > 0
        cs.append(cells[sel])
        ds.append(np.full(int(sel.sum()), a, dtype=np.int64))
        bs.append(tf[sel] - 1)
    c, d, b = np.concatenate(cs), np.concatenate(ds), np.concatenate(bs)
    order = np.lexsort((d, c))
    return c[order], d[order], b[order]


def forces_at(known, link_c, link_d, link_b, bodies, dims, periodic, tau):
    """Eq. hydroF from the deviations known at the link cells."""
    nb = neighbours(link_c, dims, periodic)
    y = nb[link_d, np.arange(link_c.size)]
    dft, rho, _ = collide_at(known, link_c, tau)
    dft_link = dft[link_d, np.arange(link_c.size)]
    return coupling.link_forces(link_d, link_b, y, dft_link, rho, bodies, dims, periodic)
