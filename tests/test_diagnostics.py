"""Diagnostics of equations (1)-(3): the oracle pinned against exact
differences and the equilibrium identities (CPU), and the GPU kernel against
the oracle element by element (GPU)."""

import numpy as np
import pytest

import synth
from oracle import diagnostics as odiag
from oracle import exact, fields


def rel(a, b):
    d = np.abs(b).max()
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / (d if d > 0 else 1.0))


def walls(shape):
    nz, ny, nx = shape
    m = np.zeros(shape, dtype=bool)
    m[:, :, 0] = m[:, :, -1] = True
    m[:, 0, :] = m[:, -1, :] = True
    m[-1] = True
    return m


def quadratic_case(shape, lengths):
    """Fields quadratic in each coordinate: every central and one-sided
    second-order difference of them is exact, so the diagnostics must equal
    the analytic curl, force residual and divergence to rounding."""
    nz, ny, nx = shape
    lx, ly, lz = lengths
    z, y, x = np.meshgrid(np.linspace(0, lz, nz), np.linspace(0, ly, ny), np.linspace(0, lx, nx), indexing="ij")
    Bx = x * x * y + z * z - x * z
    By = y * y * z + 2 * x * y - z
    Bz = x * y * z + y * y - 3 * x
    p = x * x + y * z
    rho = 1 + x
    # analytic derivatives
    dBx = (2 * x * y - z, x * x, 2 * z - x)  # d/dx, d/dy, d/dz
    dBy = (2 * y, 2 * y * z + 2 * x, y * y - 1)
    dBz = (y * z - 3, x * z + 2 * y, x * y)
    dp = (2 * x, z, y)
    return (x, y, z), (Bx, By, Bz, p, rho), (dBx, dBy, dBz, dp)


@pytest.mark.parametrize("shape,lengths,mu0,g", [((9, 9, 9), (1.0, 1.0, 1.0), 1.0, 1.0),
                                                  ((9, 17, 5), (1.0, 0.7, 0.4), 0.5, 2.0)])
def test_oracle_exact_on_quadratics(shape, lengths, mu0, g):
    _, (Bx, By, Bz, p, rho), (dBx, dBy, dBz, dp) = quadratic_case(shape, lengths)
    jx, jy, jz, fres, divb = odiag.diagnostics(Bx, By, Bz, p, rho, mu0, g, *lengths)
    ex = (dBz[1] - dBy[2]) / mu0
    ey = (dBx[2] - dBz[0]) / mu0
    ez = (dBy[0] - dBx[1]) / mu0
    Fx = ey * Bz - ez * By - dp[0]
    Fy = ez * Bx - ex * Bz - dp[1]
    Fz = ex * By - ey * Bx - dp[2] - rho * g
    want = (ex, ey, ez, np.sqrt(Fx**2 + Fy**2 + Fz**2), dBx[0] + dBy[1] + dBz[2])
    w = walls(Bx.shape)
    for got, ref in zip((jx, jy, jz, fres, divb), want):
        assert rel(got[~w], ref[~w]) < 1e-12
        assert np.all(got[w] == 0.0)


def smooth_case(n, a=0.6, h=0.3, alpha=0.5):
    grid = synth.make_grid(n)
    model = synth.make_model(grid, alpha, a, h)
    x = np.linspace(0, 1, n)
    bz = (np.sin(np.pi * x)[None] * np.sin(np.pi * x)[:, None]
          + 0.5 * np.sin(2 * np.pi * x)[None] * np.sin(np.pi * x)[:, None])
    bz[0] = bz[-1] = 0
    bz[:, 0] = bz[:, -1] = 0
    P = exact.solve(bz, n, model.xi, model.alpha)
    F = fields.fields(P, model.alpha, model.xi, model.dxi, model.pb, model.rhob, model.mu0, model.g)
    return model, F


def test_current_identity_order2():
    """Equation (4) with F = xi Bz / g: mu0 j = alpha B + grad(xi Bz) x e_z,
    i.e. (mu0 j - alpha B) = (d(xi Bz)/dy, -d(xi Bz)/dx, 0), to O(h^2)."""
    errs = []
    for n in (17, 33, 65):
        # a slowly varying xi (scale height 1) keeps the three grids in the
        # asymptotic range of the third derivatives this identity involves
        model, (Bx, By, Bz, p, rho) = smooth_case(n, a=0.3, h=1.0)
        jx, jy, jz, _, _ = odiag.diagnostics(Bx, By, Bz, p, rho, model.mu0, model.g)
        h = 1.0 / (n - 1)
        xb = model.xi[:, None, None] * Bz
        cy = np.zeros_like(xb)
        cx = np.zeros_like(xb)
        cy[:, 1:-1] = (xb[:, 2:] - xb[:, :-2]) / (2 * h)
        cx[:, :, 1:-1] = (xb[:, :, 2:] - xb[:, :, :-2]) / (2 * h)
        inner = (slice(2, -2),) * 3
        e = max(np.abs((model.mu0 * jx - model.alpha * Bx - cy)[inner]).max(),
                np.abs((model.mu0 * jy - model.alpha * By + cx)[inner]).max(),
                np.abs((model.mu0 * jz - model.alpha * Bz)[inner]).max())
        errs.append(e / np.abs(model.alpha * Bz[inner]).max())
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.6
    assert errs[-1] < 1e-2


def test_force_and_divergence_residuals_order2():
    """(1) and (3) hold for the continuum fields: the discrete residuals of
    a converged equilibrium fall as h^2 (relative to |j x B| and |dBx/dx|)."""
    fe, de = [], []
    for n in (17, 33, 65):
        model, (Bx, By, Bz, p, rho) = smooth_case(n)
        jx, jy, jz, fres, divb = odiag.diagnostics(Bx, By, Bz, p, rho, model.mu0, model.g)
        inner = (slice(2, -2),) * 3
        lor = np.sqrt((jy * Bz - jz * By) ** 2 + (jz * Bx - jx * Bz) ** 2 + (jx * By - jy * Bx) ** 2)[inner].max()
        fe.append(fres[inner].max() / lor)
        h = 1.0 / (n - 1)
        scale = np.abs((Bx[:, :, 2:] - Bx[:, :, :-2]) / (2 * h)).max()
        de.append(np.abs(divb[inner]).max() / scale)
    assert fe[0] / fe[1] > 3.5 and fe[1] / fe[2] > 3.5 and fe[-1] < 1e-2
    assert de[0] / de[1] > 3.5 and de[1] / de[2] > 3.5 and de[-1] < 1e-2


def test_force_free_residual_vanishes_with_xi_zero():
    """xi = 0: p = p_b, rho = rho_b (hydrostatic) and j parallel to B, so the
    residual is only the truncation error of the background balance and of
    j x B: small against |j| |B| and falling with h."""
    r = []
    for n in (33, 65):
        model, (Bx, By, Bz, p, rho) = smooth_case(n, a=0.0)
        jx, jy, jz, fres, divb = odiag.diagnostics(Bx, By, Bz, p, rho, model.mu0, model.g)
        inner = (slice(2, -2),) * 3
        jb = (np.sqrt(jx**2 + jy**2 + jz**2) * np.sqrt(Bx**2 + By**2 + Bz**2))[inner].max()
        r.append(fres[inner].max() / jb)
    assert r[0] < 0.1 and r[1] < r[0] / 2.5


# --------------------------------------------------------------------- GPU
torch = pytest.importorskip("torch")


@pytest.mark.gpu
@pytest.mark.parametrize("shape,lengths,seed", [((33, 33, 33), (1.0, 1.0, 1.0), 1),
                                               ((65, 129, 33), (1.0, 1.3, 0.6), 2),
                                               ((129, 65, 257), (0.8, 0.8, 1.0), 3)])
def test_gpu_diagnostics_match_oracle(shape, lengths, seed):
    """Random fields (every node, walls included, so wall handling is
    checked) through the kernel vs the oracle, element by element."""
    from paper_1307_6720_amd.solver import Plan, diagnostics

    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    arrs = [rng.standard_normal((nz, ny, nx)) for _ in range(5)]
    arrs[4] = np.abs(arrs[4]) + 0.5
    mu0, g = 0.5, 1.7
    model = synth.make_model(synth.make_grid(nx, ny, nz, *lengths), 0.3, 0.2, 0.3)
    model = synth.Model(model.alpha, model.xi, model.dxi, model.pb, model.rhob, mu0, g)
    want = odiag.diagnostics(*arrs, mu0, g, *lengths)
    plan = Plan(synth.make_grid(nx, ny, nz, *lengths), device="cuda:0")
    dev = [torch.from_numpy(a).to("cuda:0") for a in arrs]
    print(f"[diag] shape={shape} seed={seed}", flush=True)
    got = diagnostics(plan, model, *dev)
    torch.cuda.synchronize()
    plan.close()
    for name, gt, w in zip(("jx", "jy", "jz", "fres", "divb"), got, want):
        gt = gt.cpu().numpy()
        assert rel(gt, w) < 1e-13, (name, rel(gt, w))
        assert np.all(gt[walls(gt.shape)] == 0.0), name


@pytest.mark.gpu
def test_gpu_diagnostics_of_a_solved_equilibrium():
    """The 129^3 workload through the whole GPU path, then the diagnostics:
    the GPU kernel equals the oracle on the GPU fields, and the residuals of
    (1) and (3) are at the truncation level of the grid."""
    from paper_1307_6720_amd import PREC_MIXED
    from paper_1307_6720_amd.solver import Plan, diagnostics, solve

    w = synth.workload("mhs-129")
    m = w.model
    plan = Plan(w.grid, device="cuda:0")
    res = solve(plan, torch.from_numpy(w.bz0).to("cuda:0"), m, precision=PREC_MIXED, rtol=1e-10)
    F = (res.Bx, res.By, res.Bz, res.p, res.rho)
    got = [t.cpu().numpy() for t in diagnostics(plan, m, *F)]
    torch.cuda.synchronize()
    Fh = [t.cpu().numpy() for t in F]
    plan.close()
    want = odiag.diagnostics(*Fh, m.mu0, m.g, w.grid.lx, w.grid.ly, w.grid.lz)
    for gt, wt in zip(got, want):
        assert rel(gt, wt) < 1e-13
    jx, jy, jz, fres, divb = got
    Bx, By, Bz = Fh[:3]
    inner = (slice(2, -2),) * 3
    lor = np.sqrt((jy * Bz - jz * By) ** 2 + (jz * Bx - jx * Bz) ** 2 + (jx * By - jy * Bx) ** 2)[inner].max()
    assert fres[inner].max() < 0.05 * lor
