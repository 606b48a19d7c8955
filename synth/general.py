"""Seeded inputs of the general problem a(x) lap u + b(x) u = c(x).

Smooth coefficients varying along every axis of the grid: a = 1 + 0.5
sin(x + 2y [+ 3z]) > 0 and b = -(1 + x^2) - 5 w^2 <= 0, with w the last
axis (z in the box, the face's second axis on a face); c and the boundary
values of u are normal random numbers from numpy.random.default_rng(seed),
drawn in that order; the interior of u (the initial guess) is zero.
"""

from __future__ import annotations

import numpy as np


def general_problem(shape, lengths, seed):
    """(a, b, c, u) on a grid of `shape` ((nz, ny, nx) or (n2, n1), first
    axis slowest) over a box of `lengths` (x first)."""
    rng = np.random.default_rng(seed)
    axes = [np.linspace(0.0, L, n) for n, L in zip(shape[::-1], lengths)]
    grids = np.meshgrid(*axes[::-1], indexing="ij")  # slowest axis first
    s = sum((q + 1) * g for q, g in enumerate(grids[::-1]))
    a = 1.0 + 0.5 * np.sin(s)
    b = -(1.0 + grids[-1] ** 2) - 5.0 * grids[0] ** 2
    c = rng.normal(size=shape)
    u = rng.normal(size=shape)
    u[tuple(slice(1, -1) for _ in shape)] = 0.0
    return a, b, c, u
