"""Pins of the oracle against facts fixed by the paper and by mathematics.

Every check here compares an oracle routine with something other than itself:
closed forms of the discrete or continuum problem, brute-force dense solves,
the paper's printed relaxation formula, textbook routines (scipy's banded
solver) and identities of central differences.  Each is chosen so that a
plausible mistake (a dropped term, a wrong sign, a wrong index, a transposed
operand) fails at least one of them.
"""

import numpy as np
import pytest
from scipy.linalg import solve_banded

import synth
from oracle import dense, exact, fields, ref


def rel(a, b):
    d = np.abs(b).max()
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / (d if d > 0 else 1.0))


def mode2(nx, ny, m, n, lx=1.0, ly=1.0):
    return synth.fourier_mode(nx, ny, lx, ly, m, n)


def lam_mn(nx, ny, m, n, lx=1.0, ly=1.0):
    dx, dy = lx / (nx - 1), ly / (ny - 1)
    return (4 / dx**2) * np.sin(m * np.pi * dx / (2 * lx)) ** 2 + (4 / dy**2) * np.sin(n * np.pi * dy / (2 * ly)) ** 2


# ---------------------------------------------------------------- grid rules
def test_level_count_rule():
    # x and y halve at every step; z halves too unless dz^2 >= 2 max(dx, dy)^2;
    # stop when an axis to be halved has 3 nodes
    assert ref.levels3(3, 3, 3) == (1, [])
    assert ref.levels3(33, 33, 33) == (5, [0, 0, 0, 0])
    assert ref.nlevels3(257, 257, 257) == 8
    # dz = 2 dx: 513^2 x 257 -> 257^3 -> ... -> 3^3
    assert ref.levels3(513, 513, 257) == (9, [1, 0, 0, 0, 0, 0, 0, 0])
    assert ref.levels3(129, 129, 65) == (7, [1, 0, 0, 0, 0, 0])
    # equal spacing by the box lengths: no semicoarsening
    assert ref.levels3(129, 129, 65, (1.0, 1.0, 0.5)) == (6, [0] * 5)
    # dz = 4 dx: two steps keep z, then 5^3 -> 3^3
    assert ref.levels3(17, 17, 5) == (4, [1, 1, 0])
    # the larger in-plane spacing decides: dx = 1/64, dy = 1/32, dz = 1/16
    assert ref.levels3(65, 33, 17) == (5, [1, 0, 0, 0])
    # dz = 1.25 dx (< sqrt 2): all axes halve
    assert ref.levels3(33, 33, 33, (1.0, 1.0, 1.25))[1] == [0, 0, 0, 0]
    # x and y kept while 2 dz^2 <= min(dx, dy)^2: dz = dx / 64 halves z six
    # times (257 -> 5 nodes, dz = dx), then all axes once
    assert ref.levels3(5, 5, 257) == (8, [2, 2, 2, 2, 2, 2, 0])
    assert ref.levels3(9, 9, 129) == (7, [2, 2, 2, 2, 0, 0])
    # the smaller in-plane spacing decides: dx = 1/4, dy = 1/16, dz = 1/64
    assert ref.levels3(5, 17, 65)[1][:2] == [2, 2]
    assert ref.levels3(5, 17, 17)[1][0] == 0  # dz = dy: 2 dz^2 > dy^2
    assert ref.levels3(5, 17, 17, (1.0, 1.0, 0.6))[1][0] == 2  # dz = 0.6 dy (< 1/sqrt 2)
    assert ref.nlevels2(513, 513) == 9
    assert ref.nlevels3(30, 33, 33) < 0  # not 2^L + 1


# ---------------------------------------------------------------- equation (11)
@pytest.mark.parametrize("nx,ny,m,n,lx,ly", [(17, 17, 1, 1, 1.0, 1.0), (33, 17, 3, 2, 1.0, 1.0),
                                              (65, 65, 5, 7, 11.0, 11.0), (9, 33, 2, 9, 2.0, 0.5)])
def test_boundary_single_mode_exact(nx, ny, m, n, lx, ly):
    """A sine mode is an eigenvector of the five-point operator, so
    P0 = Bz0 / lam_mn exactly."""
    bz = mode2(nx, ny, m, n, lx, ly)
    want = bz / lam_mn(nx, ny, m, n, lx, ly)
    assert rel(exact.solve_boundary(bz, lx, ly), want) < 1e-13
    P0, st, cyc, rr = ref.mg2(bz, rtol=1e-14, lengths=(lx, ly))
    assert st == ref.OK
    assert rel(P0, want) < 1e-12


@pytest.mark.parametrize("nx,ny", [(9, 9), (17, 17), (33, 33), (17, 9)])
def test_boundary_dense_bruteforce(nx, ny):
    rng = np.random.default_rng(nx * 100 + ny)
    bz = rng.normal(size=(ny, nx))
    bz[0] = bz[-1] = 0
    bz[:, 0] = bz[:, -1] = 0
    want = dense.solve2(bz, 1.3, 0.7)
    assert rel(exact.solve_boundary(bz, 1.3, 0.7), want) < 1e-12
    P0, st, _, _ = ref.mg2(bz, rtol=1e-14, lengths=(1.3, 0.7))
    assert st == ref.OK
    assert rel(P0, want) < 1e-11


def test_boundary_given_edges():
    """P given on the edges of the base (the summary of Section 5 leaves P on
    the side boundaries to the problem): bilinear data with Bz0 = 0 is
    reproduced exactly (every
    second difference of a bilinear function vanishes), and random edges
    with a random magnetogram match the dense solve."""
    ny, nx = 17, 33
    y, x = np.meshgrid(np.linspace(0, 0.7, ny), np.linspace(0, 1.0, nx), indexing="ij")
    u = 0.3 + 1.2 * x - 0.7 * y + 2.1 * x * y
    bc = u.copy()
    bc[1:-1, 1:-1] = 0.0
    got, st, _, _ = ref.mg2(np.zeros_like(u), rtol=1e-14, lengths=(1.0, 0.7), P0=bc, keep_edges=True)
    assert st == ref.OK and rel(got, u) < 1e-12
    assert rel(dense.solve2(np.zeros_like(u), 1.0, 0.7, edges=u), u) < 1e-13
    rng = np.random.default_rng(6)
    bz = rng.normal(size=(9, 17))
    e = rng.normal(size=(9, 17))
    want = dense.solve2(bz, 1.0, 1.0, edges=e)
    e[1:-1, 1:-1] = 0.0
    got, st, _, _ = ref.mg2(bz, rtol=1e-14, P0=e, keep_edges=True)
    assert st == ref.OK and rel(got, want) < 1e-11
    # the default still zeroes the edges
    got0, _, _, _ = ref.mg2(bz, rtol=1e-14, P0=e)
    assert rel(got0, dense.solve2(bz)) < 1e-11


def test_interior_given_faces():
    """P given on every face (the summary leaves the other boundary
    conditions to the problem): with
    alpha = 0 a trilinear P satisfies (8) exactly for any xi (its second
    differences vanish), so the solve returns it; random faces match the
    dense solve."""
    shape, lengths = (17, 9, 33), (1.0, 0.8, 1.3)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.linspace(0, lengths[2], nz), np.linspace(0, lengths[1], ny),
                          np.linspace(0, lengths[0], nx), indexing="ij")
    u = 1.0 + x - 2 * y + 0.5 * z + x * y - y * z + 3 * x * z + x * y * z
    xi = 0.9 * np.exp(-np.linspace(0, 1, nz) / 0.2)
    bc = u.copy()
    bc[1:-1, 1:-1, 1:-1] = 0.0
    got, st, _, _ = ref.mg3(bc, xi, 0.0, rtol=1e-14, lengths=lengths)
    assert st == ref.OK and rel(got, u) < 1e-11
    rng = np.random.default_rng(12)
    shape = (9, 9, 17)
    bc = rng.normal(size=shape)
    bc[1:-1, 1:-1, 1:-1] = 0.0
    xi = rng.uniform(0, 0.8, 9)
    want = dense.solve3(bc, None, xi, 0.6)
    got, st, _, _ = ref.mg3(bc, xi, 0.6, rtol=1e-14)
    assert st == ref.OK and rel(got, want) < 1e-11


def test_boundary_paper_jacobi_fixed_point():
    """Iterating the paper's printed lower-boundary Jacobi update (Section 4)
    reaches the oracle's solution of (11): this pins the sign convention of
    the right-hand side (the update adds +Bz and divides by 2(1/dx^2+1/dy^2))."""
    nx = ny = 9
    bz = synth.bipolar_magnetogram(nx, ny, 1.0, 1.0, 1, np.random.default_rng(3), sigma=0.25)
    P = np.zeros_like(bz)
    for _ in range(3000):
        P = ref.jacobi2(P, bz)
    assert rel(P, exact.solve_boundary(bz)) < 1e-12


def test_boundary_continuum_order2():
    """Continuum: Bz0 = sin(pi x) sin(2 pi y) gives P0 = Bz0 / (pi^2 + 4 pi^2);
    the discrete error must fall as h^2."""
    errs = []
    for n in (17, 33, 65):
        bz = mode2(n, n, 1, 2)
        errs.append(rel(exact.solve_boundary(bz), bz / (5 * np.pi**2)))
    assert 3.8 < errs[0] / errs[1] < 4.2 and 3.8 < errs[1] / errs[2] < 4.2


# ---------------------------------------------------------------- equation (8)
def sinh_profile(nz, lz, lam, alpha):
    """Closed form of the discrete z-problem for xi = 0:
    Z_{k+1} + Z_{k-1} = (2 + dz^2 (lam - alpha^2)) Z_k, Z_0 = 1, Z_{nz-1} = 0,
    solved by sinh(kappa (lz - z_k)) / sinh(kappa lz) with
    cosh(kappa dz) = 1 + dz^2 (lam - alpha^2) / 2."""
    dz = lz / (nz - 1)
    kappa = np.arccosh(1 + dz**2 * (lam - alpha**2) / 2) / dz
    z = np.arange(nz) * dz
    return np.sinh(kappa * (lz - z)) / np.sinh(kappa * lz)


@pytest.mark.parametrize("n,m,k,alpha,lz", [(17, 1, 1, 0.0, 1.0), (33, 2, 3, 0.9, 1.0),
                                             (33, 1, 2, 2.5, 2.0), (65, 4, 1, 0.5, 1.0)])
def test_interior_single_mode_xi0_closed_form(n, m, k, alpha, lz):
    nz = n
    bz = mode2(n, n, m, k)
    lam = lam_mn(n, n, m, k)
    Z = sinh_profile(nz, lz, lam, alpha)
    want = (bz / lam)[None, :, :] * Z[:, None, None]
    xi = np.zeros(nz)
    assert rel(exact.solve(bz, nz, xi, alpha, lz=lz), want) < 1e-12
    ubc = np.zeros((nz, n, n))
    ubc[0] = bz / lam
    P, st, _, _ = ref.mg3(ubc, xi, alpha, rtol=1e-14, lengths=(1.0, 1.0, lz))
    assert st == ref.OK
    assert rel(P, want) < 1e-11


@pytest.mark.parametrize("nz,a,h,alpha", [(17, 0.7, 0.2, 0.4), (33, 0.95, 0.1, 1.0), (65, 0.5, 0.3, 0.0)])
def test_interior_single_mode_general_xi(nz, a, h, alpha):
    """For one horizontal mode, (8) reduces to a tridiagonal problem in z with
    diagonal -2/dz^2 + alpha^2 - (1 - xi_k) lam; solved here with scipy's
    banded solver as the textbook routine."""
    n = 17
    m, k = 2, 1
    bz = mode2(n, n, m, k)
    lam = lam_mn(n, n, m, k)
    z = np.linspace(0, 1, nz)
    xi = a * np.exp(-z / h)
    dz = 1.0 / (nz - 1)
    K = nz - 2
    ab = np.zeros((3, K))
    ab[0, 1:] = 1 / dz**2
    ab[2, :-1] = 1 / dz**2
    ab[1] = -2 / dz**2 + alpha**2 - (1 - xi[1:-1]) * lam
    rhs = np.zeros(K)
    rhs[0] = -1 / dz**2
    Z = np.concatenate([[1.0], solve_banded((1, 1), ab, rhs), [0.0]])
    want = (bz / lam)[None] * Z[:, None, None]
    assert rel(exact.solve(bz, nz, xi, alpha), want) < 1e-12
    ubc = np.zeros((nz, n, n))
    ubc[0] = bz / lam
    # nz = 65 over 17 x 17 is strongly anisotropic: point smoothing is slow
    P, st, _, _ = ref.mg3(ubc, xi, alpha, rtol=1e-14, max_cycles=400)
    assert st == ref.OK
    assert rel(P, want) < 1e-11


def test_interior_continuum_order2():
    """Force-free single mode in the continuum: with Bz0 = sin(pi x) sin(pi y),
    P = Bz0 sinh(kappa (1 - z)) / (sinh(kappa) k^2), k^2 = 2 pi^2,
    kappa = sqrt(k^2 - alpha^2); error must fall as h^2."""
    alpha = 0.8
    k2 = 2 * np.pi**2
    kappa = np.sqrt(k2 - alpha**2)
    errs = []
    for n in (17, 33, 65):
        bz = mode2(n, n, 1, 1)
        z = np.linspace(0, 1, n)
        want = (bz / k2)[None] * (np.sinh(kappa * (1 - z)) / np.sinh(kappa))[:, None, None]
        errs.append(rel(exact.solve(bz, n, np.zeros(n), alpha), want))
    assert 3.7 < errs[0] / errs[1] < 4.3 and 3.7 < errs[1] / errs[2] < 4.3


@pytest.mark.parametrize("shape,lengths", [((5, 5, 5), (1, 1, 1)), ((9, 9, 9), (1.0, 2.0, 0.5)),
                                           ((5, 9, 17), (1, 1, 1)), ((17, 17, 17), (11.0, 11.0, 12.0))])
def test_interior_dense_bruteforce(shape, lengths):
    nz, ny, nx = shape
    lx, ly, lz = lengths
    rng = np.random.default_rng(sum(shape))
    xi = rng.uniform(0.0, 0.9, size=nz)
    alpha = 0.3
    ubc = np.zeros(shape)
    ubc[0, 1:-1, 1:-1] = rng.normal(size=(ny - 2, nx - 2))
    want = dense.solve3(ubc, None, xi, alpha, lx, ly, lz)
    assert rel(exact.solve_interior(ubc[0], nz, xi, alpha, lx, ly, lz), want) < 1e-12
    P, st, _, _ = ref.mg3(ubc, xi, alpha, rtol=1e-14, lengths=lengths)
    assert st == ref.OK
    assert rel(P, want) < 1e-11
    # the direct solver of the oracle's coarsest level agrees too
    assert rel(ref.direct3(ubc, None, xi, alpha, lengths), want) < 1e-11


@pytest.mark.parametrize("shape,lengths", [((5, 5, 5), (1.0, 1.0, 1.0)), ((9, 9, 9), (1.0, 2.0, 0.5)),
                                           ((17, 9, 5), (1.0, 1.0, 1.0)), ((9, 17, 5), (0.7, 1.3, 2.0))])
def test_min_eigenvalue_bound_equals_dense_spectrum(shape, lengths):
    """Definiteness of (8) (Section 2.1: xi < 1 makes the operator elliptic;
    alpha^2 must stay below the spectrum).  The per-mode tridiagonal
    eigenvalue equals the smallest eigenvalue of the dense matrix
    -[(1 - xi)(d2x + d2y) + d2z] built node by node (alpha = 0), for random
    xi < 1 including values close to 1; and alpha^2 just below it leaves
    the dense operator negative definite, just above it does not."""
    nz, ny, nx = shape
    lx, ly, lz = lengths
    rng = np.random.default_rng(7 * nz + ny)
    xi = rng.uniform(-0.5, 0.98, size=nz)
    A, _ = dense.operator3(shape, xi, 0.0, lx, ly, lz)
    assert np.allclose(A, A.T, rtol=0, atol=0)
    lam_dense = np.linalg.eigvalsh(-A)
    lam0 = exact.min_eigenvalue_bound(nx, ny, nz, xi, lx, ly, lz)
    assert abs(lam0 - lam_dense[0]) <= 1e-12 * lam_dense[-1]
    for s, definite in ((1 - 1e-6, True), (1 + 1e-6, False)):
        Aa, _ = dense.operator3(shape, xi, np.sqrt(s * lam0), lx, ly, lz)
        assert (np.linalg.eigvalsh(Aa)[-1] < 0) == definite


def test_interior_with_source_dense():
    """Nonzero right-hand side and boundary data together (the form the
    coarse levels and the refinement inner solve see)."""
    shape = (9, 9, 9)
    rng = np.random.default_rng(5)
    xi = np.linspace(0.5, 0.0, 9)
    f = rng.normal(size=shape)
    ubc = np.zeros(shape)
    ubc[0] = rng.normal(size=(9, 9))
    ubc[:, 0, :] = rng.normal(size=(9, 9))
    want = dense.solve3(ubc, f, xi, 1.1)
    assert rel(ref.direct3(ubc, f, xi, 1.1), want) < 1e-12
    u = ubc.copy()
    for _ in range(30):
        u = ref.vcycle3_once(u, f, xi, 1.1)
    assert rel(u, want) < 1e-12


def test_mg_matches_exact_33_65():
    for n in (33, 65):
        w = synth.workload("mhs-129", dims=(n, n, n))
        m = w.model
        P, st, info = ref.solve(w.bz0, m.xi, m.alpha, w.grid.shape, rtol2=1e-14, rtol3=1e-14)
        assert st == ref.OK
        assert rel(P, exact.solve(w.bz0, n, m.xi, m.alpha)) < 1e-11


def test_thread_count_does_not_change_the_oracle():
    """The OpenMP loops of the C multigrid (used for the all-core CPU
    timing) compute every node as the serial loops do and split no sum, so
    the iterates are bitwise the same for any thread count (grids with
    steps that halve every axis and steps that keep z)."""
    for dims in ((33, 33, 33), (65, 33, 17)):
        w = synth.workload("mhs-129", dims=dims)
        m = w.model
        got = []
        prev = ref.set_threads(0)  # 0 leaves the count unchanged
        for th in (1, 3):
            ref.set_threads(th)
            P, st, info = ref.solve(w.bz0, m.xi, m.alpha, w.grid.shape, rtol2=1e-12, rtol3=1e-12)
            assert st == ref.OK
            got.append((P, info["cycles3d"]))
        ref.set_threads(prev)
        assert got[0][1] == got[1][1]
        assert np.array_equal(got[0][0], got[1][0])


# ---------------------------------------------------------------- multigrid stages
def trilinear_field(shape, seed):
    rng = np.random.default_rng(seed)
    c = rng.normal(size=8)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.linspace(0, 1, nz), np.linspace(0, 1, ny), np.linspace(0, 1, nx), indexing="ij")
    return (c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * y * z + c[6] * x * z
            + c[7] * x * y * z)


def test_restriction_reproduces_trilinear():
    """Full weighting has weights summing to one and symmetric first moments
    per axis, so it maps a trilinear field to its coarse-node values."""
    f = trilinear_field((17, 9, 33), 1)
    fc = ref.restrict3(f)
    want = f[::2, ::2, ::2]
    assert rel(fc[1:-1, 1:-1, 1:-1], want[1:-1, 1:-1, 1:-1]) < 1e-14
    assert np.all(fc[0] == 0) and np.all(fc[:, :, -1] == 0)
    f2 = trilinear_field((3, 17, 9), 2)[1]
    assert rel(ref.restrict2(f2)[1:-1, 1:-1], f2[::2, ::2][1:-1, 1:-1]) < 1e-14


def test_restriction_weights_point_response():
    """A unit residual at fine node (i, j, k) = (3, 4, 5) feeds the coarse
    nodes I in {1, 2}, J = 2, K in {2, 3} with w(a)w(b)w(c) = 1/4 * 1/2 * 1/4,
    w = (1/4, 1/2, 1/4) by offset -1, 0, +1."""
    rf = np.zeros((9, 9, 9))
    rf[5, 4, 3] = 1.0  # [k, j, i]
    fc = ref.restrict3(rf)
    w = 0.25 * 0.5 * 0.25
    for K, J, I in ((2, 2, 1), (2, 2, 2), (3, 2, 1), (3, 2, 2)):
        assert fc[K, J, I] == pytest.approx(w, abs=0)
    assert fc.sum() == pytest.approx(4 * w, abs=1e-17)


def test_prolongation_reproduces_trilinear():
    ec = trilinear_field((9, 5, 17), 3)
    ec[0] = ec[-1] = 0
    ec[:, 0] = ec[:, -1] = 0
    ec[:, :, 0] = ec[:, :, -1] = 0
    uf = ref.prolong3(ec, np.zeros((17, 9, 33)))
    # compare with an independent evaluation: linear interpolation per axis via numpy.interp
    zc, yc, xc = (np.linspace(0, 1, s) for s in ec.shape)
    zf, yf, xf = (np.linspace(0, 1, s) for s in uf.shape)
    t = np.apply_along_axis(lambda v: np.interp(xf, xc, v), 2, ec)
    t = np.apply_along_axis(lambda v: np.interp(yf, yc, v), 1, t)
    t = np.apply_along_axis(lambda v: np.interp(zf, zc, v), 0, t)
    assert rel(uf[1:-1, 1:-1, 1:-1], t[1:-1, 1:-1, 1:-1]) < 1e-14
    assert np.all(uf[0] == 0) and np.all(uf[:, -1] == 0)


def test_plane_restriction_is_2d_full_weighting_per_plane():
    """With z kept, the restriction is the pinned 2D full weighting applied to
    each interior plane (zero on the bottom and top planes), so it also maps
    a field bilinear in x and y to its coarse-node values."""
    rng = np.random.default_rng(4)
    rf = rng.normal(size=(7, 17, 9))
    fc = ref.restrict3_xy(rf)
    assert fc.shape == (7, 9, 5)
    for k in range(1, 6):
        assert rel(fc[k], ref.restrict2(rf[k])) < 1e-15
    assert np.all(fc[0] == 0) and np.all(fc[-1] == 0)
    f = trilinear_field((7, 17, 9), 5)
    fc = ref.restrict3_xy(f)
    assert rel(fc[1:-1, 1:-1, 1:-1], f[1:-1, ::2, ::2][:, 1:-1, 1:-1]) < 1e-14
    # point response: weights 1/4 * 1/2 (offsets +-1 in x, 0 in y), one plane
    rf = np.zeros((5, 9, 9))
    rf[2, 4, 3] = 1.0
    fc = ref.restrict3_xy(rf)
    assert fc[2, 2, 1] == 0.125 and fc[2, 2, 2] == 0.125 and fc.sum() == 0.25


def test_plane_prolongation_is_bilinear_per_plane():
    ec = trilinear_field((7, 5, 9), 6)
    ec[0] = ec[-1] = 0
    ec[:, 0] = ec[:, -1] = 0
    ec[:, :, 0] = ec[:, :, -1] = 0
    uf = ref.prolong3_xy(ec, np.zeros((7, 9, 17)))
    yc, xc = (np.linspace(0, 1, s) for s in ec.shape[1:])
    yf, xf = (np.linspace(0, 1, s) for s in uf.shape[1:])
    t = np.apply_along_axis(lambda v: np.interp(xf, xc, v), 2, ec)
    t = np.apply_along_axis(lambda v: np.interp(yf, yc, v), 1, t)
    assert rel(uf[1:-1, 1:-1, 1:-1], t[1:-1, 1:-1, 1:-1]) < 1e-14
    assert np.all(uf[0] == 0) and np.all(uf[-1] == 0) and np.all(uf[:, :, 0] == 0)


def test_z_restriction_and_prolongation_act_along_z():
    """With x and y kept, the restriction is the 1D full weighting along z
    of each column (zero on the coarse boundary) and the prolongation is
    linear interpolation along z (numpy.interp), exact on data linear in
    z."""
    rng = np.random.default_rng(8)
    rf = rng.normal(size=(17, 6, 7))
    fc = ref.restrict3_z(rf)
    assert fc.shape == (9, 6, 7)
    want = np.zeros_like(fc)
    want[1:-1, 1:-1, 1:-1] = (0.25 * rf[1:-3:2] + 0.5 * rf[2:-2:2] + 0.25 * rf[3:-1:2])[:, 1:-1, 1:-1]
    assert rel(fc, want) < 1e-15
    f = trilinear_field((17, 6, 7), 9)
    assert rel(ref.restrict3_z(f)[1:-1, 1:-1, 1:-1], f[::2][1:-1, 1:-1, 1:-1]) < 1e-14
    ec = trilinear_field((9, 5, 6), 10)
    ec[0] = ec[-1] = 0
    ec[:, 0] = ec[:, -1] = 0
    ec[:, :, 0] = ec[:, :, -1] = 0
    uf = ref.prolong3_z(ec, np.zeros((17, 5, 6)))
    zc, zf = np.linspace(0, 1, 9), np.linspace(0, 1, 17)
    t = np.apply_along_axis(lambda v: np.interp(zf, zc, v), 0, ec)
    assert rel(uf[1:-1, 1:-1, 1:-1], t[1:-1, 1:-1, 1:-1]) < 1e-14
    assert np.all(uf[:, 0] == 0) and np.all(uf[0] == 0) and np.all(uf[-1] == 0)


def test_residual_matches_dense_matrix():
    shape = (5, 9, 7 + 2)
    rng = np.random.default_rng(9)
    xi = rng.uniform(0, 0.8, shape[0])
    u = rng.normal(size=shape)
    f = rng.normal(size=shape)
    A, bnd = dense.operator3(shape, xi, 0.6)
    Au = A @ u[1:-1, 1:-1, 1:-1].reshape(-1)
    for r, w, idx in bnd:
        Au[r] += w * u[idx]
    want = f[1:-1, 1:-1, 1:-1].reshape(-1) - Au
    got = ref.residual3(u, f, xi, 0.6)
    assert rel(got[1:-1, 1:-1, 1:-1].reshape(-1), want) < 1e-13
    assert np.all(got[0] == 0) and np.all(got[:, :, 0] == 0)


def test_rbgs_matches_sequential_row_solves():
    """One red-black sweep equals solving each red row of the dense system in
    turn, then each black row, using the latest values."""
    shape = (7, 5, 9)
    nz, ny, nx = shape
    rng = np.random.default_rng(11)
    xi = rng.uniform(0, 0.8, nz)
    alpha = 0.9
    u0 = rng.normal(size=shape)
    f = rng.normal(size=shape)
    A, bnd = dense.operator3(shape, xi, alpha)
    shift = np.zeros(A.shape[0])
    for r, w, idx in bnd:
        shift[r] += w * u0[idx]
    x = u0[1:-1, 1:-1, 1:-1].reshape(-1).copy()
    b = f[1:-1, 1:-1, 1:-1].reshape(-1) - shift
    idx = [(i, j, k) for k in range(1, nz - 1) for j in range(1, ny - 1) for i in range(1, nx - 1)]
    for colour in (0, 1):
        for r, (i, j, k) in enumerate(idx):
            if (i + j + k) % 2 == colour:
                x[r] = (b[r] - (A[r] @ x - A[r, r] * x[r])) / A[r, r]
    got = ref.rbgs3(u0, f, xi, alpha, 1)
    assert rel(got[1:-1, 1:-1, 1:-1].reshape(-1), x) < 1e-13
    assert np.array_equal(got[0], u0[0]) and np.array_equal(got[:, :, -1], u0[:, :, -1])


def _vcycle_from_stages(u, f, xi, alpha, lengths, nu1=2, nu2=2):
    """V-cycle assembled from the separately pinned stages: red-black
    smoothing, residual, full weighting, a zero initial coarse guess, xi
    sampled at coarse nodes (xi_{l+1}[k] = xi_l[2k]), doubled spacing, an
    exact dense solve on the coarsest grid and trilinear prolongation; on a
    step that keeps z (dz^2 >= 2 max(dx, dy)^2) the transfers act within
    planes and xi is not resampled."""
    nz, ny, nx = u.shape
    hx, hy, hz = lengths[0] / (nx - 1), lengths[1] / (ny - 1), lengths[2] / (nz - 1)
    kind = "xy" if hz * hz >= 2.0 * max(hx, hy) ** 2 else "z" if 2.0 * hz * hz <= min(hx, hy) ** 2 else "all"
    if (kind != "z" and (nx <= 3 or ny <= 3)) or (kind != "xy" and nz <= 3):
        return dense.solve3(u, f, xi, alpha, *lengths)
    u = ref.rbgs3(u, f, xi, alpha, nu1, lengths)
    r = ref.residual3(u, f, xi, alpha, lengths)
    restrict = {"xy": ref.restrict3_xy, "z": ref.restrict3_z, "all": ref.restrict3}[kind]
    prolong = {"xy": ref.prolong3_xy, "z": ref.prolong3_z, "all": ref.prolong3}[kind]
    fc = restrict(r)
    ec = _vcycle_from_stages(np.zeros_like(fc), fc, xi if kind == "xy" else xi[::2], alpha, lengths, nu1, nu2)
    return ref.rbgs3(prolong(ec, u), f, xi, alpha, nu2, lengths)


@pytest.mark.parametrize("shape,lengths", [((5, 9, 9), (1.0, 1.5, 0.75)), ((17, 17, 9), (1.0, 1.5, 0.75)),
                                           ((9, 17, 33), (1.0, 1.5, 0.75)), ((9, 17, 33), (1.0, 1.0, 1.0)),
                                           ((5, 17, 17), (1.0, 1.0, 1.0)), ((33, 5, 9), (1.0, 1.0, 1.0)),
                                           ((65, 9, 5), (1.0, 1.0, 1.0))])
def test_vcycle_equals_composition_of_stages(shape, lengths):
    rng = np.random.default_rng(len(shape) + shape[0])
    nz = shape[0]
    xi = 0.9 * np.exp(-np.linspace(0, 1, nz) / 0.15)
    u0 = rng.normal(size=shape)
    f = rng.normal(size=shape)
    want = _vcycle_from_stages(u0, f, xi, 0.7, lengths)
    got = ref.vcycle3_once(u0, f, xi, 0.7, lengths=lengths)
    assert rel(got, want) < 1e-12


def _vcycle2_from_stages(u, f, nu1=2, nu2=2):
    if min(u.shape) <= 3:
        # one interior unknown per row/column at most: exact dense solve
        A = dense.operator2(u.shape)
        x = np.linalg.solve(A, f[1:-1, 1:-1].reshape(-1))
        out = u.copy()
        out[1:-1, 1:-1] = x.reshape(u.shape[0] - 2, u.shape[1] - 2)
        return out
    u = ref.rbgs2(u, f, nu1)
    fc = ref.restrict2(ref.residual2(u, f))
    ec = _vcycle2_from_stages(np.zeros_like(fc), fc, nu1, nu2)
    return ref.rbgs2(ref.prolong2(ec, u), f, nu2)


def test_boundary_cycle_equals_composition_of_stages():
    """One cycle of the oracle's lower-boundary multigrid equals the cycle
    assembled from its pinned 2D stages (f = -Bz0, zero initial guess)."""
    bz = synth.bipolar_magnetogram(33, 17, 1.0, 1.0, 2, np.random.default_rng(8), sigma=0.1)
    f = -bz
    f[0] = f[-1] = 0
    f[:, 0] = f[:, -1] = 0
    want = _vcycle2_from_stages(np.zeros_like(bz), f)
    got, st, cyc, rr = ref.mg2(bz, rtol=0.0, max_cycles=1)
    assert cyc == 1
    assert rel(got, want) < 1e-13


def test_vcycle_contraction_poisson():
    """V(2,2) with red-black smoothing and full weighting contracts the
    residual of 3D Poisson by roughly 0.1 per cycle; a broken transfer or a
    mis-scaled coarse right-hand side pushes this toward 1."""
    n = 33
    rng = np.random.default_rng(2)
    ubc = np.zeros((n, n, n))
    ubc[0, 1:-1, 1:-1] = rng.normal(size=(n - 2, n - 2))
    P, st, cyc, rr, hist = ref.mg3(ubc, np.zeros(n), 0.0, rtol=1e-12, history=True)
    rates = hist[3:] / hist[2:-1]
    assert rates.max() < 0.2


def test_vcycle_contraction_with_dz_much_below_dx():
    """dz = dx / 32 (9 x 9 x 257): halving z alone until the spacing is
    equal keeps the cycle contracting (below 0.15 per cycle); halving every
    axis leaves point smoothing unable to reduce the error along z and the
    cycle barely contracts."""
    nz, n = 257, 9
    xi = 0.5 * np.exp(-np.linspace(0.0, 1.0, nz) / 0.3)
    rng = np.random.default_rng(5)
    ubc = np.zeros((nz, n, n))
    ubc[0, 1:-1, 1:-1] = rng.normal(size=(n - 2, n - 2))
    P, st, cyc, rr, hist = ref.mg3(ubc, xi, 0.3, rtol=1e-12, history=True)
    assert st == ref.OK
    assert (hist[3:] / hist[2:-1]).max() < 0.15
    assert rel(P, exact.solve_interior(ubc[0], nz, xi, 0.3, 1.0, 1.0, 1.0)) < 1e-9


def test_vcycle_contraction_with_dz_twice_dx():
    """dz = 2 dx with xi -> 1 at the base (the strongly anisotropic large
    case): halving x and y alone first keeps the cycle contracting as on an
    equally spaced grid (below 0.15 per cycle); coarsening all three axes
    together would leave every level anisotropic (about 0.26 per cycle
    here)."""
    nz, n = 33, 65
    z = np.linspace(0.0, 1.0, nz)
    xi = np.exp(-z / 0.1)
    rng = np.random.default_rng(4)
    ubc = np.zeros((nz, n, n))
    ubc[0, 1:-1, 1:-1] = rng.normal(size=(n - 2, n - 2))
    P, st, cyc, rr, hist = ref.mg3(ubc, xi, 0.8, rtol=1e-12, history=True)
    assert st == ref.OK
    rates = hist[3:] / hist[2:-1]
    assert rates.max() < 0.15, rates
    assert rel(P, exact.solve_interior(ubc[0], nz, xi, 0.8, 1.0, 1.0, 1.0)) < 1e-9


# ---------------------------------------------------------------- fields
def test_fields_single_mode_closed_form():
    """For P = A sin(kx x) sin(ky y) Z_k, the central differences have closed
    forms, e.g. D_x sin(kx x) = sin(kx dx)/dx cos(kx x); this pins every term
    and sign of Bx, By, Bz."""
    n, nz = 17, 17
    m, k = 2, 1
    alpha = 0.7
    bz = mode2(n, n, m, k)
    lam = lam_mn(n, n, m, k)
    Z = sinh_profile(nz, 1.0, lam, alpha)
    P = (bz / lam)[None] * Z[:, None, None]
    Bx, By, Bz = fields.magnetic_field(P, alpha)
    h = 1.0 / (n - 1)
    x = np.linspace(0, 1, n)
    kx, ky = m * np.pi, k * np.pi
    sx, cx = np.sin(kx * x)[None, None, :], np.cos(kx * x)[None, None, :]
    sy, cy = np.sin(ky * x)[None, :, None], np.cos(ky * x)[None, :, None]
    Dx, Dy = np.sin(kx * h) / h, np.sin(ky * h) / h
    dZ = np.zeros(nz)
    dZ[1:-1] = (Z[2:] - Z[:-2]) / (2 * h)
    dZ[0] = (-3 * Z[0] + 4 * Z[1] - Z[2]) / (2 * h)
    A = 1 / lam
    Zc, dZc = Z[:, None, None], dZ[:, None, None]
    wBx = A * (alpha * sx * Dy * cy * Zc + Dx * cx * sy * dZc)
    wBy = A * (-alpha * Dx * cx * sy * Zc + sx * Dy * cy * dZc)
    wBz = lam * A * sx * sy * Zc
    inner = (slice(0, -1), slice(1, -1), slice(1, -1))
    for got, want in ((Bx, wBx), (By, wBy), (Bz, wBz)):
        assert rel(got[inner], want[inner]) < 1e-12
        assert np.all(got[-1] == 0) and np.all(got[:, 0] == 0) and np.all(got[:, :, -1] == 0)
    # Bz on the base reproduces the prescribed magnetogram
    assert rel(Bz[0, 1:-1, 1:-1], bz[1:-1, 1:-1]) < 1e-13


def smooth_case(n, a=0.5, h=0.3, alpha=0.5):
    grid = synth.make_grid(n)
    model = synth.make_model(grid, alpha, a, h)
    x = np.linspace(0, 1, n)
    bz = (np.sin(np.pi * x)[None] * np.sin(np.pi * x)[:, None]
          + 0.5 * np.sin(2 * np.pi * x)[None] * np.sin(np.pi * x)[:, None])
    bz[0] = bz[-1] = 0
    bz[:, 0] = bz[:, -1] = 0
    P = exact.solve(bz, n, model.xi, model.alpha)
    return grid, model, bz, P


def central(a, axis, h):
    out = np.zeros_like(a)
    s = [slice(None)] * 3
    s[axis] = slice(1, -1)
    p = [slice(None)] * 3
    p[axis] = slice(2, None)
    q = [slice(None)] * 3
    q[axis] = slice(None, -2)
    out[tuple(s)] = (a[tuple(p)] - a[tuple(q)]) / (2 * h)
    return out


def test_divergence_free_wide_stencil_identity():
    """Central differences commute, so with the wide-stencil
    Bz~ = -(D_x^2 + D_y^2) P the discrete divergence D_x Bx + D_y By + D_z Bz~
    vanishes to rounding away from the walls; this pins the alpha terms and
    the mixed derivatives of Bx and By (equation (5) with T = alpha P)."""
    n = 33
    grid, model, bz, P = smooth_case(n)
    Bx, By, Bz = fields.magnetic_field(P, model.alpha)
    h = 1.0 / (n - 1)
    Bzw = -(central(central(P, 2, h), 2, h) + central(central(P, 1, h), 1, h))
    div = central(Bx, 2, h) + central(By, 1, h) + central(Bzw, 0, h)
    inner = (slice(2, -2),) * 3
    scale = np.abs(central(Bx, 2, h)[inner]).max()
    assert np.abs(div[inner]).max() < 1e-11 * scale


def test_force_free_curl_equals_alpha_b():
    """xi = 0 makes the field linear force-free: curl B = alpha B, to O(h^2)."""
    errs = []
    for n in (17, 33, 65):
        grid, model, bz, P = smooth_case(n, a=0.0, alpha=0.9)
        Bx, By, Bz = fields.magnetic_field(P, model.alpha)
        h = 1.0 / (n - 1)
        jx = central(Bz, 1, h) - central(By, 0, h)
        jy = central(Bx, 0, h) - central(Bz, 2, h)
        jz = central(By, 2, h) - central(Bx, 1, h)
        inner = (slice(2, -2),) * 3
        e = max(np.abs((jx - model.alpha * Bx)[inner]).max(), np.abs((jy - model.alpha * By)[inner]).max(),
                np.abs((jz - model.alpha * Bz)[inner]).max())
        errs.append(e / np.abs(model.alpha * Bz[inner]).max())
    assert errs[-1] < 1.5e-2
    assert errs[0] / errs[1] > 2.9 and errs[1] / errs[2] > 3.4


def test_force_balance_order2():
    """Equation (1): (curl B) x B / mu0 - grad p - rho g e_z = 0 with p, rho
    from (9) and (10) and a background in hydrostatic balance; the discrete
    residual must fall as h^2 relative to |j x B|."""
    errs = []
    for n in (17, 33, 65):
        grid, model, bz, P = smooth_case(n, a=0.6, h=0.3, alpha=0.5)
        Bx, By, Bz, p, rho = fields.fields(P, model.alpha, model.xi, model.dxi, model.pb, model.rhob,
                                           model.mu0, model.g)
        h = 1.0 / (n - 1)
        jx = central(Bz, 1, h) - central(By, 0, h)
        jy = central(Bx, 0, h) - central(Bz, 2, h)
        jz = central(By, 2, h) - central(Bx, 1, h)
        Fx = (jy * Bz - jz * By) / model.mu0 - central(p, 2, h)
        Fy = (jz * Bx - jx * Bz) / model.mu0 - central(p, 1, h)
        Fz = (jx * By - jy * Bx) / model.mu0 - central(p, 0, h) - rho * model.g
        # the background balances to O(h^2) too; remove the analytic part
        inner = (slice(2, -2),) * 3
        lor = np.sqrt(((jy * Bz - jz * By) ** 2 + (jz * Bx - jx * Bz) ** 2 + (jx * By - jy * Bx) ** 2)[inner]).max()
        res = np.sqrt((Fx**2 + Fy**2 + Fz**2)[inner]).max()
        errs.append(res / lor)
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5
    assert errs[-1] < 1e-2


def test_pressure_density_equal_background_when_xi_zero():
    n = 17
    grid, model, bz, P = smooth_case(n, a=0.0)
    Bx, By, Bz, p, rho = fields.fields(P, model.alpha, model.xi, model.dxi, model.pb, model.rhob)
    assert np.array_equal(p, np.broadcast_to(model.pb[:, None, None], p.shape))
    assert np.array_equal(rho, np.broadcast_to(model.rhob[:, None, None], rho.shape))


def test_pressure_deficit_sign():
    """Equation (9): positive xi lowers the pressure where Bz is strong."""
    grid, model, bz, P = smooth_case(17, a=0.5)
    Bx, By, Bz, p, rho = fields.fields(P, model.alpha, model.xi, model.dxi, model.pb, model.rhob)
    dp = p - model.pb[:, None, None]
    assert dp.max() <= 0.0 and dp.min() < 0.0
    k, j, i = 3, 8, 5
    assert dp[k, j, i] == pytest.approx(-model.xi[k] * Bz[k, j, i] ** 2 / 2.0, rel=1e-15)


def test_base_bz_equals_magnetogram():
    w = synth.workload("potential-33")
    m = w.model
    P = exact.solve(w.bz0, 33, m.xi, m.alpha)
    _, _, Bz = fields.magnetic_field(P, m.alpha)
    assert rel(Bz[0, 1:-1, 1:-1], w.bz0[1:-1, 1:-1]) < 1e-12


# ---------------------------------------------------------------- inputs
def test_magnetogram_zero_flux_and_reproducible():
    for name in ("potential-33", "mhs-129"):
        a = synth.workload(name, dims=(65, 65, 65)).bz0
        b = synth.workload(name, dims=(65, 65, 65)).bz0
        assert np.array_equal(a, b)
        assert abs(a[1:-1, 1:-1].sum()) < 1e-14 * np.abs(a).sum()
        assert np.all(a[0] == 0) and np.all(a[:, -1] == 0)
    w = synth.workload("mhs-513x513x257", dims=(65, 65, 33))
    assert abs(w.bz0[1:-1, 1:-1].sum()) < 1e-13 * np.abs(w.bz0).sum()


def test_paper_three_source_magnetogram():
    """Section 3.1: sources of width l = 0.3, +1 at (1.5, 1.5) and -0.5 at
    (-1.5, -1.5) and (1.5, -1.5), on [-5.5, 5.5]^2 (node spacing 11/128)."""
    n = 129
    srcs = [(1.5, 1.5, 1.0), (-1.5, -1.5, -0.5), (1.5, -1.5, -0.5)]
    bz = synth.gaussian_sources(n, n, 11.0, 11.0, srcs, 0.3, x0=-5.5, y0=-5.5)
    x = -5.5 + np.arange(n) * 11.0 / (n - 1)
    jmax, imax = np.unravel_index(np.argmax(bz), bz.shape)
    assert abs(x[imax] - 1.5) < 11.0 / 128 and abs(x[jmax] - 1.5) < 11.0 / 128
    assert 0.9 < bz.max() <= 1.0
    assert -0.5 <= bz.min() < -0.45
    neg = bz < -0.25
    assert neg[:, x < 0].any() and neg[x < 0, :].any()
