"""The interior solve without allocation (mhs_solve_interior_noalloc)
against the plan-based mhs_solve_interior on the same inputs.

Both run the same kernels with the same tiling, so P must agree bitwise
(the parity bar of the solve path is 1e-10 relative for FP64 and 1e-8 for
the mixed path; bitwise is stricter).  Calls follow each other on one
device with shrinking grids, so the second and third calls find the
previous call's contents in the shared scratch array; the largest grid the
array holds (129^3) is the first call; a grid past it (257^3)
is refused on the host (tests/test_abi.py).  Each solve is also checked against the exact discrete
solution, so that both paths are right, not only equal.
"""

import numpy as np
import pytest

import synth
from oracle import exact

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1307_6720_amd import PREC_FP64, PREC_MIXED  # noqa: E402
from paper_1307_6720_amd.solver import Plan, make_opts, solve_interior_noalloc  # noqa: E402

DEV = torch.device("cuda:0")


def rel(a, b):
    d = np.abs(b).max()
    return float(np.abs(a - b).max() / (d if d > 0 else 1.0))


def base_plane(w):
    """P with plane 0 from the plan-based boundary solve (rtol 1e-13)."""
    plan = Plan(w.grid, PREC_FP64, device=DEV)
    P = torch.zeros(w.grid.shape, dtype=torch.float64, device=DEV)
    plan.solve_boundary(torch.from_numpy(w.bz0).to(DEV), P, make_opts(rtol=1e-13))
    torch.cuda.synchronize()
    plan.close()
    return P


def test_noalloc_matches_plan_path():
    # 129^3 mixed (the largest workspace the scratch array holds), then a
    # smaller FP64 grid, then a smaller anisotropic mixed grid
    cases = [((129, 129, 129), PREC_MIXED, 1e-10, 1e-8),
             ((65, 65, 65), PREC_FP64, 1e-12, 1e-10),
             ((65, 33, 17), PREC_MIXED, 1e-10, 1e-8)]
    for dims, prec, rtol, tol in cases:
        print(f"[noalloc] {dims} precision {prec}", flush=True)
        w = synth.workload("mhs-129", dims=dims)
        m = w.model
        P0 = base_plane(w)
        plan = Plan(w.grid, prec, device=DEV)
        Pa = P0.clone()
        ia = plan.solve_interior(m, Pa, make_opts(prec, rtol))
        Pb = P0.clone()
        ib = solve_interior_noalloc(w.grid, m, Pb, make_opts(prec, rtol))
        torch.cuda.synchronize()
        plan.close()
        assert ia.status == 0 and ib.status == 0
        assert ib.cycles == ia.cycles and ib.inner_cycles == ia.inner_cycles
        assert ib.rel_residual == ia.rel_residual and ib.r0 == ia.r0
        assert torch.equal(Pa, Pb), float((Pa - Pb).abs().max())
        want = exact.solve(w.bz0, w.grid.nz, m.xi, m.alpha, w.grid.lx, w.grid.ly, w.grid.lz)
        err = rel(Pb.cpu().numpy(), want)
        print(f"[noalloc] {dims} cycles {ib.cycles} error {err:.2e}", flush=True)
        assert err < tol, err
