"""Magnetic field lines of a recovered equilibrium.

ORACLE -- test infrastructure, not the product.

Section 3 presents each equilibrium through its field lines (curves tangent
to B, e.g. the lines that reach the base near a null); the paper does not
say how they are traced.  The reading taken here:

  * a line through a seed x0 solves  dx/ds = B(x) / |B(x)|  in arc length
    s; a negative step ds traces against B;
  * B between nodes is the trilinear interpolation of the node values of
    the cell that holds the point, evaluated as nested linear
    interpolations a + t (b - a): along x on the cell's four x-edges, then
    along y, then along z; a point outside the box [0, lx] x [0, ly] x
    [0, lz] takes the value at its coordinates clamped to the box;
  * the classical fourth-order Runge-Kutta method with the fixed step ds:
        k1 = T(x),  k2 = T(x + (ds/2) k1),  k3 = T(x + (ds/2) k2),
        k4 = T(x + ds k3),  x' = x + (ds/6) (((k1 + 2 k2) + 2 k3) + k4),
    T = B / |B| with |B| = sqrt((Bx^2 + By^2) + Bz^2) and each component
    divided by |B|;
  * a line ends when a step would leave the box (status EXIT; that point is
    not kept), when a stage finds |B| <= bmin (status NULL, near a
    magnetic null), or after max_steps steps (status MAXSTEPS).  A seed
    outside the box is a line of one point with status EXIT.

Lines are advanced together with numpy over the lines still running; every
operation is elementwise, so each line is computed exactly as it would be
on its own.
"""

from __future__ import annotations

import numpy as np

MAXSTEPS, EXIT, NULL = 0, 1, 2


def sample(F, pos, lengths):
    """Trilinear interpolation of the (nz, ny, nx) node array F at the
    points pos (m, 3) = (x, y, z), coordinates clamped to the box."""
    F = np.asarray(F, dtype=np.float64)
    nz, ny, nx = F.shape
    n = (nx, ny, nz)
    cell = []
    for a in range(3):
        h = lengths[a] / (n[a] - 1)
        p = np.minimum(np.maximum(pos[:, a], 0.0), lengths[a])
        f = p / h
        i = np.minimum(np.floor(f).astype(np.int64), n[a] - 2)
        cell.append((i, f - i))
    (i, tx), (j, ty), (k, tz) = cell

    def lerp(a, b, t):
        return a + t * (b - a)

    c00 = lerp(F[k, j, i], F[k, j, i + 1], tx)
    c10 = lerp(F[k, j + 1, i], F[k, j + 1, i + 1], tx)
    c01 = lerp(F[k + 1, j, i], F[k + 1, j, i + 1], tx)
    c11 = lerp(F[k + 1, j + 1, i], F[k + 1, j + 1, i + 1], tx)
    return lerp(lerp(c00, c10, ty), lerp(c01, c11, ty), tz)


def _tangent(B, pos, lengths, bmin):
    bx, by, bz = (sample(F, pos, lengths) for F in B)
    b = np.sqrt((bx * bx + by * by) + bz * bz)
    ok = b > bmin
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.stack([bx / b, by / b, bz / b], axis=1)
    # a failed stage ends the line; zero keeps the later stages finite
    return np.where(ok[:, None], t, 0.0), ok


def _inside(pos, lengths):
    return np.all((pos >= 0.0) & (pos <= np.asarray(lengths, dtype=np.float64)), axis=1)


def trace(Bx, By, Bz, seeds, ds, max_steps, bmin=0.0, lengths=(1.0, 1.0, 1.0)):
    """Trace one field line per seed.

    Returns (points, count, status): points (max_steps + 1, nlines, 3) with
    line l's points in points[:count[l], l] (the rest zero), count >= 1
    (the seed is point 0), status MAXSTEPS, EXIT or NULL per line."""
    B = tuple(np.asarray(F, dtype=np.float64) for F in (Bx, By, Bz))
    seeds = np.asarray(seeds, dtype=np.float64).reshape(-1, 3)
    m = seeds.shape[0]
    pts = np.zeros((max_steps + 1, m, 3))
    pts[0] = seeds
    count = np.ones(m, dtype=np.int32)
    status = np.full(m, MAXSTEPS, dtype=np.int32)
    run = _inside(seeds, lengths)
    status[~run] = EXIT
    x = seeds.copy()
    hh, h6 = 0.5 * ds, ds / 6.0
    for n in range(max_steps):
        idx = np.nonzero(run)[0]
        if idx.size == 0:
            break
        p = x[idx]
        k1, ok1 = _tangent(B, p, lengths, bmin)
        k2, ok2 = _tangent(B, p + hh * k1, lengths, bmin)
        k3, ok3 = _tangent(B, p + hh * k2, lengths, bmin)
        k4, ok4 = _tangent(B, p + ds * k3, lengths, bmin)
        null = ~(ok1 & ok2 & ok3 & ok4)
        q = p + h6 * (((k1 + 2.0 * k2) + 2.0 * k3) + k4)
        out = ~null & ~_inside(q, lengths)
        step = ~null & ~out
        status[idx[null]] = NULL
        status[idx[out]] = EXIT
        run[idx[null | out]] = False
        good = idx[step]
        x[good] = q[step]
        pts[n + 1, good] = q[step]
        count[good] += 1
    return pts, count, status
