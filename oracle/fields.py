"""Recovery of B, p and rho from the poloidal potential P.

ORACLE -- test infrastructure, not the product.

Section 2.2 gives, with T = alpha P (equation (6)) in equation (5),
    Bx = alpha dP/dy + d2P/dxdz,
    By = -alpha dP/dx + d2P/dydz,
    Bz = -(d2P/dx2 + d2P/dy2)            (the operator of equation (11)),
approximated by second-order central differences, then
    p   = p_b - xi Bz^2 / (2 mu0)                                   (9)
    rho = rho_b + (xi' Bz^2/(2 mu0) + xi (B . grad Bz)/mu0) / g       (10)
with the derivatives of Bz in (10) again by central differences.

Boundary reading (the paper does not say how faces are treated): B = 0 on
the side and top faces, as the walls of Section 2.2 assume; on the base
(k = 0) the z-derivatives are the second-order one-sided difference
(-3 f_0 + 4 f_1 - f_2) / (2 dz), and Bz uses the same in-plane five-point
stencil as in the interior.  On faces where B = 0, p = p_b and rho = rho_b.
"""

from __future__ import annotations

import numpy as np


def _dcentral(a, axis, h):
    """Central difference (a[+1] - a[-1]) / (2h) along ``axis``; NaN at the
    two end nodes, where it is undefined."""
    out = np.full_like(a, np.nan)
    n = a.shape[axis]
    c = [slice(None)] * a.ndim
    p = [slice(None)] * a.ndim
    m = [slice(None)] * a.ndim
    c[axis] = slice(1, n - 1)
    p[axis] = slice(2, n)
    m[axis] = slice(0, n - 2)
    out[tuple(c)] = (a[tuple(p)] - a[tuple(m)]) / (2.0 * h)
    return out


def _dz_with_base(a, dz):
    """d/dz: central at 1..nz-2, one-sided second order at k = 0."""
    out = _dcentral(a, 0, dz)
    out[0] = (-3.0 * a[0] + 4.0 * a[1] - a[2]) / (2.0 * dz)
    return out


def _second(a, axis, h):
    """(a[+1] - 2a + a[-1]) / h^2 along ``axis``; NaN at the end nodes."""
    out = np.full_like(a, np.nan)
    n = a.shape[axis]
    c = [slice(None)] * a.ndim
    p = [slice(None)] * a.ndim
    m = [slice(None)] * a.ndim
    c[axis] = slice(1, n - 1)
    p[axis] = slice(2, n)
    m[axis] = slice(0, n - 2)
    out[tuple(c)] = (a[tuple(p)] - 2.0 * a[tuple(c)] + a[tuple(m)]) / (h * h)
    return out


def _wall_mask(shape):
    """True on the side faces and the top face (where B = 0)."""
    nz, ny, nx = shape
    m = np.zeros(shape, dtype=bool)
    m[:, :, 0] = m[:, :, -1] = True
    m[:, 0, :] = m[:, -1, :] = True
    m[-1, :, :] = True
    return m


def magnetic_field(P, alpha, lx=1.0, ly=1.0, lz=1.0):
    """Return (Bx, By, Bz) on every node, shape (nz, ny, nx)."""
    P = np.asarray(P, dtype=np.float64)
    nz, ny, nx = P.shape
    dx, dy, dz = lx / (nx - 1), ly / (ny - 1), lz / (nz - 1)
    walls = _wall_mask(P.shape)
    dzP = _dz_with_base(P, dz)
    Bx = alpha * _dcentral(P, 1, dy) + _dcentral(dzP, 2, dx)
    By = -alpha * _dcentral(P, 2, dx) + _dcentral(dzP, 1, dy)
    Bz = -(_second(P, 2, dx) + _second(P, 1, dy))
    for B in (Bx, By, Bz):
        B[walls] = 0.0
    return Bx, By, Bz


def fields(P, alpha, xi, dxi, pb, rhob, mu0=1.0, g=1.0, lx=1.0, ly=1.0, lz=1.0):
    """Return (Bx, By, Bz, p, rho) on every node."""
    P = np.asarray(P, dtype=np.float64)
    nz, ny, nx = P.shape
    dx, dy, dz = lx / (nx - 1), ly / (ny - 1), lz / (nz - 1)
    Bx, By, Bz = magnetic_field(P, alpha, lx, ly, lz)
    xi3 = np.asarray(xi, dtype=np.float64)[:, None, None]
    dxi3 = np.asarray(dxi, dtype=np.float64)[:, None, None]
    pb3 = np.asarray(pb, dtype=np.float64)[:, None, None]
    rhob3 = np.asarray(rhob, dtype=np.float64)[:, None, None]
    p = pb3 - xi3 * Bz * Bz / (2.0 * mu0)
    dBzx = _dcentral(Bz, 2, dx)
    dBzy = _dcentral(Bz, 1, dy)
    dBzz = _dz_with_base(Bz, dz)
    rho = rhob3 + (dxi3 * Bz * Bz / (2.0 * mu0)
                   + xi3 * (Bx * dBzx + By * dBzy + Bz * dBzz) / mu0) / g
    walls = _wall_mask(P.shape)
    p = np.where(walls, np.broadcast_to(pb3, P.shape), p)
    rho = np.where(walls, np.broadcast_to(rhob3, P.shape), rho)
    return Bx, By, Bz, p, rho
