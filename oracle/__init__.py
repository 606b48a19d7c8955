"""ORACLE -- test infrastructure, not the product.

Plain, slow, obviously correct FP64 CPU implementations of what the solver
computes, written from Section 2.2 of MacTaggart et al. (arXiv:1307.6720):

* ``exact``  -- the exact solution of the two discrete elliptic systems,
  equations (11) and (8), by sine transforms in x, y and a tridiagonal solve
  per mode in z (the discrete operator separates because xi depends on z
  only and alpha is constant).
* ``ref``    -- ctypes binding of ``mg_ref.c``: the same V(2,2) multigrid
  method as the HIP path, in plain C loops (the algorithmic twin).
* ``fields`` -- recovery of B, p and rho by central differences
  (Section 2.2, equations (5), (6), (9), (10)).
* ``dense``  -- brute-force dense solves on tiny grids.
* ``diagnostics`` -- current density, force-balance and divergence residuals
  of equations (1)-(3) (Section 2.1) by the same differences.
* ``fieldlines`` -- magnetic field lines (the curves Section 3 draws):
  fourth-order Runge-Kutta in arc length on trilinearly interpolated B.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path
(``paper_1307_6720_amd``); both take their inputs from ``synth``.
"""
