"""Diagnostics of a recovered equilibrium: current density, force balance and
divergence of B.

ORACLE -- test infrastructure, not the product.

Section 2.1 states the MHS equations the equilibrium satisfies:
    (1)  mu0^-1 (curl B) x B - grad p - rho g e_z = 0,
    (2)  curl B = mu0 j,
    (3)  div B = 0.
Given B, p and rho on the grid (from the field recovery of Section 2.2), the
diagnostics evaluate, with second-order central differences,
    j    = (curl B) / mu0                                (2)
    F    = j x B - grad p - rho g e_z                    (the residual of (1))
    fres = |F|
    divb = d Bx/dx + d By/dy + d Bz/dz                   (the residual of (3))
A converged equilibrium has F and divb of order h^2 (the continuous fields
satisfy (1) and (3) exactly; the discrete ones to the truncation error).

Reading (the paper gives no stencil for these): the same differences as the
field recovery -- central in x, y and in z above the base, the one-sided
second-order difference (-3 f0 + 4 f1 - f2) / (2 dz) at k = 0.  On the side
faces and the top face, where B is set to zero, every diagnostic is zero.
"""

from __future__ import annotations

import numpy as np

from .fields import _dcentral, _dz_with_base, _wall_mask


def diagnostics(Bx, By, Bz, p, rho, mu0=1.0, g=1.0, lx=1.0, ly=1.0, lz=1.0):
    """Return (jx, jy, jz, fres, divb), each of shape (nz, ny, nx)."""
    Bx, By, Bz, p, rho = (np.asarray(a, dtype=np.float64) for a in (Bx, By, Bz, p, rho))
    nz, ny, nx = Bx.shape
    dx, dy, dz = lx / (nx - 1), ly / (ny - 1), lz / (nz - 1)

    def ddx(a):
        return _dcentral(a, 2, dx)

    def ddy(a):
        return _dcentral(a, 1, dy)

    def ddz(a):
        return _dz_with_base(a, dz)

    # (2): mu0 j = curl B
    jx = (ddy(Bz) - ddz(By)) / mu0
    jy = (ddz(Bx) - ddx(Bz)) / mu0
    jz = (ddx(By) - ddy(Bx)) / mu0
    # (1): residual of the force balance
    Fx = (jy * Bz - jz * By) - ddx(p)
    Fy = (jz * Bx - jx * Bz) - ddy(p)
    Fz = (jx * By - jy * Bx) - ddz(p) - rho * g
    fres = np.sqrt(Fx * Fx + Fy * Fy + Fz * Fz)
    # (3)
    divb = ddx(Bx) + ddy(By) + ddz(Bz)
    walls = _wall_mask(Bx.shape)
    out = []
    for a in (jx, jy, jz, fres, divb):
        a = a.copy()
        a[walls] = 0.0
        out.append(a)
    return tuple(out)
