"""Pins of the oracle's general elliptic solver (Section 2.2's form
a(x) lap u + b(x) u = c(x), u given on the boundary), against facts that do
not come from the oracle's multigrid itself:

* the dense solve of the undivided form on tiny grids (3D and a face);
* a discrete eigenmode of lap_h with constant a and b (closed form);
* the exact solvers of (11) and (8) (sine transform + tridiagonal), which
  the general form reduces to for a = 1, b = 0, c = -Bz0 on a face and for
  a = 1, b = alpha^2, c = 0 in the box with the base plane as data;
* second-order convergence to a smooth solution of the continuum problem
  with variable a, b;
* invariance under scaling a, b, c by one positive function;
* the definiteness rule, the singular-a check and the fixed-cycle mode;
* each stage of the cycle (residual, red-black sweep, exact solve against
  the dense matrix; coarse b/a sampling) and one V-cycle as the
  composition of those stages on 2-, 3- and 4-level cubes, plus its
  contraction rate.
"""

import numpy as np
import pytest

import synth
from oracle import dense, exact, ref


def rel(a, b):
    d = np.abs(b).max()
    return float(np.abs(a - b).max() / (d if d > 0 else 1.0))


def random_problem(shape, seed, bscale=1.0):
    rng = np.random.default_rng(seed)
    a = 1.0 + 0.5 * rng.random(shape)
    b = -bscale * rng.random(shape)
    c = rng.normal(size=shape)
    u = rng.normal(size=shape)
    u[tuple(slice(1, -1) for _ in shape)] = rng.normal(size=tuple(n - 2 for n in shape))  # initial guess
    return a, b, c, u


@pytest.mark.parametrize("shape,lengths", [((5, 5, 5), (1.0, 1.0, 1.0)), ((9, 5, 9), (1.0, 0.5, 1.0)),
                                           ((5, 9, 17), (1.0, 0.5, 0.25)), ((17, 9, 9), (0.5, 0.5, 2.0))])
def test_general_3d_equals_dense(shape, lengths):
    a, b, c, u = random_problem(shape, 1)
    want = dense.general(a, b, c, u, lengths)
    got, st, cyc, relres, _ = ref.gen_mg(u, a, b, c, rtol=1e-13, max_cycles=80, lengths=lengths)
    assert st == ref.OK, (st, cyc, relres)
    assert rel(got, want) < 1e-11
    # boundary values are data: untouched
    inner = tuple(slice(1, -1) for _ in shape)
    mask = np.ones(shape, bool)
    mask[inner] = False
    assert np.array_equal(got[mask], u[mask])


@pytest.mark.parametrize("shape,lengths", [((9, 9), (1.0, 1.0)), ((9, 17), (2.0, 1.0)), ((17, 5), (1.0, 0.25))])
def test_general_face_equals_dense(shape, lengths):
    a, b, c, u = random_problem(shape, 2)
    want = dense.general(a, b, c, u, lengths)
    got, st, cyc, relres, _ = ref.gen_mg(u, a, b, c, rtol=1e-13, max_cycles=200, lengths=lengths, planar=True)
    assert st == ref.OK, (st, cyc, relres)
    assert rel(got, want) < 1e-11


@pytest.mark.parametrize("planar", [False, True])
def test_general_discrete_eigenmode(planar):
    """u = product of sine modes is an eigenvector of lap_h with eigenvalue
    -sum (4/h^2) sin^2(k h / 2); with constant a, b and c = (b - a lambda) u
    the solution is the mode itself (zero boundary)."""
    if planar:
        shape, lengths, modes = (17, 33), (1.0, 0.5), (3, 2)
    else:
        shape, lengths, modes = (17, 33, 17), (1.0, 0.5, 2.0), (2, 3, 1)
    axes = [np.linspace(0.0, L, n) for n, L in zip(shape[::-1], lengths)]  # x, y[, z]
    lam = 0.0
    mode = np.ones(shape)
    for ax, (x, L, m) in enumerate(zip(axes, lengths, modes)):
        h = x[1] - x[0]
        k = m * np.pi / L
        lam += 4.0 / h**2 * np.sin(k * h / 2) ** 2
        shp = [1] * len(shape)
        shp[len(shape) - 1 - ax] = -1
        mode = mode * np.sin(k * x).reshape(shp)
    a = np.full(shape, 2.5)
    b = np.full(shape, -3.0)
    c = (b - a * lam) * mode
    got, st, cyc, relres, _ = ref.gen_mg(np.zeros(shape), a, b, c, rtol=1e-14, max_cycles=100, lengths=lengths,
                                         planar=planar)
    assert st == ref.OK
    assert rel(got, mode) < 1e-12


def test_general_face_reduces_to_equation_11():
    """a = 1, b = 0, c = -Bz0 with zero edges is equation (11): the same
    solution as the sine-transform solve of the lower boundary."""
    w = synth.workload("mhs-129", dims=(33, 65, 17))
    g = w.grid
    shape = (g.ny, g.nx)
    got, st, cyc, relres, _ = ref.gen_mg(np.zeros(shape), np.ones(shape), np.zeros(shape), -w.bz0, rtol=1e-14,
                                         max_cycles=100, lengths=(g.lx, g.ly), planar=True)
    assert st == ref.OK
    want = exact.solve_boundary(w.bz0, g.lx, g.ly)
    assert rel(got, want) < 1e-12


def test_general_box_reduces_to_equation_8():
    """a = 1, b = alpha^2, c = 0 in the box, the base plane from (11) and
    zero on the other faces, is equation (8) with xi = 0: the same solution
    as the per-mode tridiagonal solve."""
    w = synth.workload("mhs-129", dims=(33, 33, 33))
    g = w.grid
    alpha = 0.8
    want = exact.solve(w.bz0, g.nz, np.zeros(g.nz), alpha, g.lx, g.ly, g.lz)
    u = np.zeros(g.shape)
    u[0] = want[0]
    shape = g.shape
    got, st, cyc, relres, _ = ref.gen_mg(u, np.ones(shape), np.full(shape, alpha**2), np.zeros(shape), rtol=1e-14,
                                         max_cycles=100, lengths=(g.lx, g.ly, g.lz))
    assert st == ref.OK
    assert rel(got, want) < 1e-11


def test_general_second_order_convergence():
    """Smooth u* with variable a > 0 and b < 0: c = a lap u* + b u* from the
    derivatives of u*, u* on the boundary; the error falls as h^2."""
    def ustar(x, y, z):
        return np.exp(x) * np.sin(2 * y) * np.cos(z) + x * y * z

    def lap(x, y, z):
        return np.exp(x) * np.sin(2 * y) * np.cos(z) * (1.0 - 4.0 - 1.0)

    errs = []
    for n in (9, 17, 33):
        z, y, x = np.meshgrid(*(np.linspace(0, 1, n),) * 3, indexing="ij")
        a = 1.0 + 0.5 * np.sin(x + 2 * y + 3 * z)
        b = -(1.0 + x**2)
        c = a * lap(x, y, z) + b * ustar(x, y, z)
        u = ustar(x, y, z)
        u[1:-1, 1:-1, 1:-1] = 0.0
        got, st, cyc, relres, _ = ref.gen_mg(u, a, b, c, rtol=1e-13, max_cycles=60)
        assert st == ref.OK
        errs.append(np.abs(got - ustar(x, y, z)).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.6 and 3.5 < r2 < 4.6, errs


def test_general_row_scaling_invariance():
    """Scaling a, b, c by one positive function leaves the discrete
    solution unchanged (each row is divided by a)."""
    shape = (9, 17, 9)
    a, b, c, u = random_problem(shape, 3)
    s = 0.2 + np.random.default_rng(4).random(shape) * 5.0
    u1, st1, *_ = ref.gen_mg(u, a, b, c, rtol=1e-14, max_cycles=80)
    u2, st2, *_ = ref.gen_mg(u, s * a, s * b, s * c, rtol=1e-14, max_cycles=80)
    assert st1 == ref.OK and st2 == ref.OK
    assert rel(u2, u1) < 1e-12


def test_general_definiteness_and_checks():
    """b/a must stay below half the smallest eigenvalue of -lap_h on the
    coarsest grid (the 3^3 grid of a cube: 3 (4/h^2) sin^2(pi/4) with
    h = 1/2, i.e. 24, so the bound is 12); a must not vanish."""
    shape = (17, 17, 17)
    a = np.ones(shape)
    c = np.ones(shape)
    u = np.zeros(shape)
    ok = ref.gen_mg(u, a, np.full(shape, 11.9), c, rtol=1e-10, max_cycles=50)
    assert ok[1] == ref.OK
    bad = ref.gen_mg(u, a, np.full(shape, 12.1), c, rtol=1e-10, max_cycles=50)
    assert bad[1] == ref.INDEFINITE
    a0 = a.copy()
    a0[8, 8, 8] = 0.0
    assert ref.gen_mg(u, a0, np.zeros(shape), c, rtol=1e-10, max_cycles=50)[1] == ref.SINGULAR
    # a vanishing a on a boundary node is not a row of the system
    a1 = a.copy()
    a1[0, 3, 3] = 0.0
    assert ref.gen_mg(u, a1, np.zeros(shape), c, rtol=1e-10, max_cycles=50)[1] == ref.OK
    # rtol < 0: exactly max_cycles cycles
    got = ref.gen_mg(u, a, np.zeros(shape), c, rtol=-1.0, max_cycles=3)
    assert got[1] == ref.OK and got[2] == 3 and len(got[4]) == 4


def test_general_levels_follow_the_rule_of_equation_8():
    """The general problem coarsens like (8): same level counts."""
    for dims, lengths in (((33, 33, 33), (1.0, 1.0, 1.0)), ((129, 129, 65), (1.0, 1.0, 1.0)),
                          ((9, 9, 129), (1.0, 1.0, 1.0)), ((65, 33, 17), (1.0, 1.0, 1.0))):
        nx, ny, nz = dims
        assert ref.gen_levels((nz, ny, nx), lengths) == ref.nlevels3(nx, ny, nz, lengths)
    assert ref.gen_levels((33, 65), (1.0, 1.0), planar=True) == ref.nlevels2(65, 33)


# ---------------------------------------------------------------- stages of the general cycle
def divided(a, b, c):
    """beta = b/a, gamma = c/a on interior nodes (zero elsewhere)."""
    inner = tuple(slice(1, -1) for _ in a.shape)
    beta, gamma = np.zeros(a.shape), np.zeros(a.shape)
    beta[inner] = b[inner] / a[inner]
    gamma[inner] = c[inner] / a[inner]
    return beta, gamma


@pytest.mark.parametrize("shape,lengths,planar", [((5, 9, 9), (1.0, 0.5, 1.0), False),
                                                  ((9, 17), (1.0, 0.5), True)])
def test_general_stages_against_the_dense_operator(shape, lengths, planar):
    """Residual, one red-black sweep and the exact solve of the divided form
    against the dense matrix of the undivided form: the residual is
    (c - A u) / a, a sweep is Gauss-Seidel over the rows of A taken red
    nodes first then black (each node solving its own row), the exact solve
    is A^-1."""
    a, b, c, u = random_problem(shape, 5)
    inner = tuple(slice(1, -1) for _ in shape)
    A, shift = dense.general_operator(a, b, u, lengths)
    beta, gamma = divided(a, b, c)
    # residual
    r, st = ref.gen_residual(u, a, b, c, lengths, planar=planar)
    want = (c[inner].reshape(-1) + shift - A @ u[inner].reshape(-1)) / a[inner].reshape(-1)
    assert st == ref.OK
    assert rel(r[inner].reshape(-1), want) < 1e-12
    mask = np.ones(shape, bool)
    mask[inner] = False
    assert not r[mask].any()
    # one sweep
    x = u[inner].reshape(-1).copy()
    rhs = c[inner].reshape(-1) + shift
    nodes = list(np.ndindex(*[n - 2 for n in shape]))
    for colour in (0, 1):
        for pos, node in enumerate(nodes):
            if sum(q + 1 for q in node) % 2 != colour:
                continue
            x[pos] = (rhs[pos] - A[pos] @ x + A[pos, pos] * x[pos]) / A[pos, pos]
    got = ref.gen_rbgs(u, beta, gamma, 1, lengths, planar=planar)
    assert rel(got[inner].reshape(-1), x) < 1e-13
    assert np.array_equal(got[mask], u[mask])
    # exact solve
    got, st = ref.gen_direct(u, beta, gamma, lengths, planar=planar)
    assert st == ref.OK
    assert rel(got, dense.general(a, b, c, u, lengths)) < 1e-12


def test_general_coarse_beta_is_sampled_at_coarse_nodes():
    rng = np.random.default_rng(6)
    beta = rng.normal(size=(9, 17, 33))
    assert np.array_equal(ref.gen_inject(beta, ref.STEP_ALL), beta[::2, ::2, ::2])
    assert np.array_equal(ref.gen_inject(beta, ref.STEP_XY), beta[:, ::2, ::2])
    assert np.array_equal(ref.gen_inject(beta, ref.STEP_Z), beta[::2])
    assert np.array_equal(ref.gen_inject(beta[0], planar=True), beta[0, ::2, ::2])


def _vcycle(u, beta, gamma, levels, nu1, nu2):
    """One V(nu1, nu2) cycle of lap_h u + beta u = gamma on cubes with every
    axis halved, composed from the separately pinned stages."""
    n = u.shape[0]
    if n == 3:
        return ref.gen_direct(u, beta, gamma)[0]
    u = ref.gen_rbgs(u, beta, gamma, nu1)
    ones = np.ones(u.shape)
    r, _ = ref.gen_residual(u, ones, beta, gamma)
    fc = ref.restrict3(r)
    bc = ref.gen_inject(beta, ref.STEP_ALL)
    ec = _vcycle(np.zeros(fc.shape), bc, fc, levels - 1, nu1, nu2)
    u = ref.prolong3(ec, u)
    return ref.gen_rbgs(u, beta, gamma, nu2)


@pytest.mark.parametrize("n", [5, 9, 17])
def test_general_vcycle_is_the_composition_of_its_stages(n):
    """One oracle V(2,2) cycle equals the cycle composed from the pinned
    stages (sweeps, residual, full weighting, coarse beta sampling,
    trilinear interpolation, the exact coarsest solve) on 2-, 3- and
    4-level cubes."""
    z, y, x = np.meshgrid(*(np.linspace(0, 1, n),) * 3, indexing="ij")
    a = 1.0 + 0.5 * np.sin(x + 2 * y + 3 * z)
    b = -(1.0 + x**2) - 20.0 * z**2
    c = np.random.default_rng(7).normal(size=a.shape)
    u = np.random.default_rng(8).normal(size=a.shape)
    beta, gamma = divided(a, b, c)
    want = _vcycle(u, beta, gamma, 0, 2, 2)
    got, st, cyc, *_ = ref.gen_mg(u, a, b, c, rtol=-1.0, max_cycles=1)
    assert st == ref.OK and cyc == 1
    assert rel(got, want) < 1e-13


def test_general_contraction():
    """V(2,2) on a 33^3 cube with a and b varying in every direction
    contracts the residual by < 0.15 per cycle (Poisson-like)."""
    n = 33
    z, y, x = np.meshgrid(*(np.linspace(0, 1, n),) * 3, indexing="ij")
    a = 1.0 + 0.5 * np.sin(x + 2 * y + 3 * z)
    b = -(1.0 + x**2) - 300.0 * z**2
    c = np.random.default_rng(0).normal(size=a.shape)
    got, st, cyc, relres, hist = ref.gen_mg(np.zeros(a.shape), a, b, c, rtol=-1.0, max_cycles=8)
    assert st == ref.OK
    assert (hist[1:] / hist[:-1]).max() < 0.15
