"""Brute-force dense solves of the discrete problems on tiny grids.

ORACLE -- test infrastructure, not the product.

Each interior node contributes one row of the seven-point form of equation
(8) (five-point form of (11) in 2D); couplings to boundary nodes move to the
right-hand side.  The dense system is solved with numpy.linalg.solve.  Only
for grids with a few thousand unknowns.
"""

from __future__ import annotations

import numpy as np


def operator3(shape, xi, alpha, lx=1.0, ly=1.0, lz=1.0):
    """Dense matrix of equation (8) over interior unknowns, plus a function
    that maps boundary data (full array) to the right-hand-side shift."""
    nz, ny, nx = shape
    dx, dy, dz = lx / (nx - 1), ly / (ny - 1), lz / (nz - 1)
    mx, my, mz = nx - 2, ny - 2, nz - 2
    m = mx * my * mz

    def row(i, j, k):
        return (i - 1) + mx * ((j - 1) + my * (k - 1))

    A = np.zeros((m, m))
    bnd = []  # (row, coefficient, (k, j, i)) couplings to boundary nodes
    for k in range(1, nz - 1):
        ax = (1.0 - xi[k]) / dx**2
        ay = (1.0 - xi[k]) / dy**2
        az = 1.0 / dz**2
        for j in range(1, ny - 1):
            for i in range(1, nx - 1):
                r = row(i, j, k)
                A[r, r] = alpha**2 - 2 * ax - 2 * ay - 2 * az
                for (a, b, c), w in (((i + 1, j, k), ax), ((i - 1, j, k), ax),
                                     ((i, j + 1, k), ay), ((i, j - 1, k), ay),
                                     ((i, j, k + 1), az), ((i, j, k - 1), az)):
                    if a in (0, nx - 1) or b in (0, ny - 1) or c in (0, nz - 1):
                        bnd.append((r, w, (c, b, a)))
                    else:
                        A[r, row(a, b, c)] += w
    return A, bnd


def solve3(u_bc, f, xi, alpha, lx=1.0, ly=1.0, lz=1.0):
    """Solve A u = f at interior nodes with boundary values from u_bc."""
    u_bc = np.asarray(u_bc, dtype=np.float64)
    A, bnd = operator3(u_bc.shape, xi, alpha, lx, ly, lz)
    rhs = np.zeros(A.shape[0]) if f is None else np.asarray(f)[1:-1, 1:-1, 1:-1].reshape(-1).copy()
    for r, w, idx in bnd:
        rhs[r] -= w * u_bc[idx]
    x = np.linalg.solve(A, rhs)
    u = u_bc.copy()
    u[1:-1, 1:-1, 1:-1] = x.reshape(u_bc.shape[0] - 2, u_bc.shape[1] - 2, u_bc.shape[2] - 2)
    return u


def operator2(shape, lx=1.0, ly=1.0):
    ny, nx = shape
    dx, dy = lx / (nx - 1), ly / (ny - 1)
    mx, my = nx - 2, ny - 2
    m = mx * my
    A = np.zeros((m, m))
    for j in range(1, ny - 1):
        for i in range(1, nx - 1):
            r = (i - 1) + mx * (j - 1)
            A[r, r] = -2.0 / dx**2 - 2.0 / dy**2
            for (a, b), w in (((i + 1, j), 1 / dx**2), ((i - 1, j), 1 / dx**2),
                              ((i, j + 1), 1 / dy**2), ((i, j - 1), 1 / dy**2)):
                if 0 < a < nx - 1 and 0 < b < ny - 1:
                    A[r, (a - 1) + mx * (b - 1)] += w
    return A


def solve2(bz0, lx=1.0, ly=1.0, edges=None):
    """Solve the five-point form of (11) with P0 = 0 on the edges, or with
    the edge values of the array `edges` (same shape) as Dirichlet data."""
    bz0 = np.asarray(bz0, dtype=np.float64)
    ny, nx = bz0.shape
    dx, dy = lx / (nx - 1), ly / (ny - 1)
    A = operator2(bz0.shape, lx, ly)
    P0 = np.zeros_like(bz0)
    rhs = -bz0[1:-1, 1:-1].copy()
    if edges is not None:
        e = np.asarray(edges, dtype=np.float64)
        P0[0], P0[-1], P0[:, 0], P0[:, -1] = e[0], e[-1], e[:, 0], e[:, -1]
        rhs[:, 0] -= P0[1:-1, 0] / dx**2
        rhs[:, -1] -= P0[1:-1, -1] / dx**2
        rhs[0, :] -= P0[0, 1:-1] / dy**2
        rhs[-1, :] -= P0[-1, 1:-1] / dy**2
    x = np.linalg.solve(A, rhs.reshape(-1))
    P0[1:-1, 1:-1] = x.reshape(ny - 2, nx - 2)
    return P0


def general_operator(a, b, u_bc, lengths=(1.0, 1.0, 1.0)):
    """Dense matrix of a lap_h + b (Section 2.2's general form, central
    differences, not divided by a) over the interior unknowns of u_bc's grid
    (3D (nz, ny, nx) or a face (ny, nx) with the lengths of its two axes),
    and the right-hand-side shift -(couplings to u_bc's boundary values)."""
    u_bc = np.asarray(u_bc, dtype=np.float64)
    nd = u_bc.ndim
    shape = u_bc.shape
    h = [l / (n - 1) for n, l in zip(shape[::-1], lengths)]  # (hx, hy[, hz])
    inner = [n - 2 for n in shape]
    idx = np.arange(int(np.prod(inner))).reshape(inner)
    m = idx.size
    A = np.zeros((m, m))
    shift = np.zeros(m)
    for node in np.ndindex(*inner):
        p = tuple(q + 1 for q in node)  # array index (k, j, i) or (j, i)
        r = idx[node]
        av = a[p]
        A[r, r] = b[p] - 2.0 * av * sum(1.0 / hh**2 for hh in h)
        for axis in range(nd):
            hh = h[nd - 1 - axis]  # array axis 0 is z (3D) or y (2D)
            for step in (-1, 1):
                q = list(p)
                q[axis] += step
                q = tuple(q)
                if 0 < q[axis] < shape[axis] - 1:
                    A[r, idx[tuple(v - 1 for v in q)]] += av / hh**2
                else:
                    shift[r] -= av / hh**2 * u_bc[q]
    return A, shift


def general(a, b, c, u_bc, lengths=(1.0, 1.0, 1.0)):
    """Exact discrete solution of a lap_h u + b u = c with u_bc's boundary
    values as Dirichlet data (shapes as general_operator)."""
    u_bc = np.asarray(u_bc, dtype=np.float64)
    nd = u_bc.ndim
    inner = tuple(slice(1, -1) for _ in range(nd))
    A, shift = general_operator(a, b, u_bc, lengths)
    x = np.linalg.solve(A, np.asarray(c, dtype=np.float64)[inner].reshape(-1) + shift)
    u = u_bc.copy()
    u[inner] = x.reshape(u[inner].shape)
    return u
