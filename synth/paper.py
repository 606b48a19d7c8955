"""The paper's own example configurations (Section 3).

Domain [-5.5, 5.5]^2 x [0, 12] with 129^3 nodes (128 intervals per axis),
B = 0 on the side and top walls, non-dimensional units in which the
magnetic pressure is |B|^2 (B0 = (2 mu0 p0)^(1/2) makes mu0 = 1/2) and
g = 1 (lengths in units of the pressure scale height).

Background atmosphere: the piecewise temperature T_b(z) of Section 3 (1 in
the photosphere/chromosphere 0 <= z <= 5, T_cor^((z-5)/5) in the transition
region, T_cor = 150 above z = 10), hydrostatic balance dp_b/dz = -p_b g/T_b
with p_b(0) = 1, and rho_b = p_b / T_b.  The balance integrates in closed
form, p_b = exp(-g I(z)) with I(z) the integral of 1/T_b from 0 to z.

Cases:
* "paper-ff": force-free (xi = 0), alpha = 0.4, three Gaussian sources of
  width l = 0.3: +1 at (1.5, 1.5), -0.5 at (-1.5, -1.5) and (1.5, -1.5);
* "paper-xi1" / "paper-xi2": the cross-field profiles
  xi_1 = 0.7 exp(-0.2 z) and xi_2 = (0.7 + 0.3 sin(pi z)) exp(-0.1 z).
  The paper names neither the magnetogram nor alpha for these runs (a
  reading): the force-free case's sources, alpha = 0.4 with xi_1 and
  alpha = 0.3 with xi_2.  With xi_2, alpha = 0.4 would sit within 4 % of the
  smallest eigenvalue of the 129^3 operator (0.1666 against 0.16), where no
  coarse grid of a few hundred unknowns still represents the lowest mode.
"""

from __future__ import annotations

import numpy as np

from .magnetogram import gaussian_sources
from .workloads import Model, Workload, make_grid

DOMAIN = (11.0, 11.0, 12.0)
ORIGIN = (-5.5, -5.5)
T_COR = 150.0
MU0 = 0.5
G = 1.0
ALPHA = 0.4
SOURCES = ((1.5, 1.5, 1.0), (-1.5, -1.5, -0.5), (1.5, -1.5, -0.5))
WIDTH = 0.3


def temperature(z, t_cor=T_COR):
    z = np.asarray(z, dtype=np.float64)
    return np.where(z <= 5.0, 1.0, np.where(z <= 10.0, t_cor ** ((z - 5.0) / 5.0), t_cor))


def background(z, g=G, t_cor=T_COR):
    """(p_b, rho_b) of the paper's atmosphere at heights z."""
    z = np.asarray(z, dtype=np.float64)
    lt = np.log(t_cor)
    zt = np.clip(z, 5.0, 10.0)
    integral = np.minimum(z, 5.0) + (5.0 / lt) * (1.0 - t_cor ** (-(zt - 5.0) / 5.0)) \
        + np.maximum(z - 10.0, 0.0) / t_cor
    p = np.exp(-g * integral)
    return p, p / temperature(z, t_cor)


def xi_profile(z, which):
    """(xi, xi') for which = "ff" (zero), "xi1" or "xi2"."""
    z = np.asarray(z, dtype=np.float64)
    if which == "ff":
        return np.zeros_like(z), np.zeros_like(z)
    if which == "xi1":
        e = np.exp(-0.2 * z)
        return 0.7 * e, -0.14 * e
    if which == "xi2":
        e = np.exp(-0.1 * z)
        s = 0.7 + 0.3 * np.sin(np.pi * z)
        return s * e, (0.3 * np.pi * np.cos(np.pi * z)) * e - 0.1 * s * e
    raise ValueError(which)


CASES = {"paper-ff": "ff", "paper-xi1": "xi1", "paper-xi2": "xi2"}


ALPHAS = {"paper-ff": ALPHA, "paper-xi1": ALPHA, "paper-xi2": 0.3}


def paper_workload(name="paper-ff", n=129, dims=None):
    """One of the paper's cases on its domain at n^3 nodes (or ``dims``)."""
    nx, ny, nz = (n, n, n) if dims is None else dims
    grid = make_grid(nx, ny, nz, *DOMAIN)
    z = grid.z()
    xi, dxi = xi_profile(z, CASES[name])
    pb, rhob = background(z)
    alpha = ALPHAS[name]
    model = Model(alpha, xi, dxi, pb, rhob, MU0, G)
    bz0 = gaussian_sources(nx, ny, DOMAIN[0], DOMAIN[1], SOURCES, WIDTH, *ORIGIN)
    return Workload(name, grid, model, bz0, 0, 1e-8, dict(alpha=alpha, xi=CASES[name], origin=ORIGIN))
