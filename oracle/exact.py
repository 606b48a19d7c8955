"""Exact solution of the discrete lower-boundary and interior problems.

ORACLE -- test infrastructure, not the product.

The multigrid method of Section 2.2 converges to the exact solution x* of
two linear systems, which this module computes directly:

* equation (11) on the base, five-point form
      (d2x + d2y) P0 = -Bz0 at interior nodes, P0 = 0 on the edges;
* equation (8) in the interior, seven-point form
      (1 - xi_k)(d2x + d2y) P + d2z P + alpha^2 P = 0 at interior nodes,
      P(., ., 0) = P0, P = 0 on the side and top faces.

With Dirichlet walls on a uniform grid, the sine vectors
sin(m*pi*i/(nx-1)) diagonalise d2x with eigenvalue
-(4/dx^2) sin^2(m*pi/(2(nx-1))) (likewise in y).  Because xi depends on z
only and alpha is a constant, each horizontal mode (m, n) decouples into a
tridiagonal problem in z:
      (Z_{k+1} - 2 Z_k + Z_{k-1})/dz^2 + (alpha^2 - (1 - xi_k) lam_mn) Z_k = 0,
      Z_0 = P0_hat(m, n),  Z_{nz-1} = 0,
solved here by plain forward elimination and back substitution.  The sine
transform is scipy's orthonormal DST-I (its own inverse).
"""

from __future__ import annotations

import numpy as np
import scipy.fft as sfft


def _lam_1d(n, h):
    """Eigenvalues of -d2 on n nodes with Dirichlet ends, modes 1..n-2."""
    m = np.arange(1, n - 1, dtype=np.float64)
    return (4.0 / (h * h)) * np.sin(m * np.pi / (2.0 * (n - 1))) ** 2


def horizontal_eigenvalues(nx, ny, lx=1.0, ly=1.0):
    """lam_mn = eigenvalue of -(d2x + d2y), shape (ny-2, nx-2)."""
    lx_ = _lam_1d(nx, lx / (nx - 1))
    ly_ = _lam_1d(ny, ly / (ny - 1))
    return ly_[:, None] + lx_[None, :]


def _dst2(a):
    return sfft.dstn(a, type=1, axes=(-2, -1), norm="ortho")


def solve_boundary(bz0, lx=1.0, ly=1.0):
    """Exact solution of the five-point form of equation (11)."""
    bz0 = np.asarray(bz0, dtype=np.float64)
    ny, nx = bz0.shape
    lam = horizontal_eigenvalues(nx, ny, lx, ly)
    bhat = _dst2(bz0[1:-1, 1:-1])
    # -(lam) P_hat = -b_hat
    P0 = np.zeros_like(bz0)
    P0[1:-1, 1:-1] = _dst2(bhat / lam)
    return P0


def _thomas_const_offdiag(off, diag, rhs):
    """Solve the tridiagonal systems off*x[k-1] + diag[k]*x[k] + off*x[k+1] = rhs[k]
    along axis 0 (all other axes are independent systems)."""
    K = diag.shape[0]
    cp = np.empty_like(diag)
    dp = np.empty_like(rhs)
    cp[0] = off / diag[0]
    dp[0] = rhs[0] / diag[0]
    for k in range(1, K):
        m = diag[k] - off * cp[k - 1]
        cp[k] = off / m
        dp[k] = (rhs[k] - off * dp[k - 1]) / m
    x = np.empty_like(rhs)
    x[K - 1] = dp[K - 1]
    for k in range(K - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


def solve_interior(P0, nz, xi, alpha, lx=1.0, ly=1.0, lz=1.0):
    """Exact solution of the seven-point form of equation (8).

    P0 is the base plane (ny, nx) with zero edges; returns P (nz, ny, nx)."""
    P0 = np.asarray(P0, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    ny, nx = P0.shape
    dz = lz / (nz - 1)
    lam = horizontal_eigenvalues(nx, ny, lx, ly)
    p0hat = _dst2(P0[1:-1, 1:-1])
    kk = np.arange(1, nz - 1)
    off = 1.0 / (dz * dz)
    diag = (-2.0 / (dz * dz) + alpha * alpha) - (1.0 - xi[kk])[:, None, None] * lam[None, :, :]
    rhs = np.zeros_like(diag)
    rhs[0] = -off * p0hat
    zhat = _thomas_const_offdiag(off, diag, rhs)
    P = np.zeros((nz, ny, nx))
    P[0] = P0
    P[1:-1, 1:-1, 1:-1] = _dst2(zhat)
    return P


def solve(bz0, nz, xi, alpha, lx=1.0, ly=1.0, lz=1.0):
    """The three steps of Section 2.2 with exact discrete solves."""
    P0 = solve_boundary(bz0, lx, ly)
    return solve_interior(P0, nz, xi, alpha, lx, ly, lz)


def min_eigenvalue_bound(nx, ny, nz, xi, lx=1.0, ly=1.0, lz=1.0):
    """Smallest eigenvalue of -[(1-xi)(d2x+d2y) + d2z] restricted to the
    interior unknowns, computed per mode from the symmetric tridiagonal
    matrices (exact, used to check definiteness for a given alpha)."""
    from scipy.linalg import eigh_tridiagonal

    xi = np.asarray(xi, dtype=np.float64)
    dz = lz / (nz - 1)
    lam = horizontal_eigenvalues(nx, ny, lx, ly)
    # the minimum over modes is attained at the smallest horizontal eigenvalue
    lmin = lam.min()
    kk = np.arange(1, nz - 1)
    d = 2.0 / (dz * dz) + (1.0 - xi[kk]) * lmin
    e = np.full(nz - 3, -1.0 / (dz * dz))
    return float(eigh_tridiagonal(d, e, eigvals_only=True)[0])
