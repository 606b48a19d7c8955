"""Solve-level parity of the HIP path against the oracle.

* algorithm parity: the HIP V-cycles and the C twin (same method, same
  stopping rule) produce the same iterates at a fixed number of cycles;
* solution parity: at the stopping tolerance, P, B, p - p_b and rho - rho_b
  match the exact discrete solution (sine transform + tridiagonal) within
  1e-10 (FP64 path) and 1e-8 (FP32-in-FP64 refinement), relative max norm
  per field;
* error paths of the C ABI.
"""

import numpy as np
import pytest

import synth
from oracle import exact, fields, ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1307_6720_amd import PREC_FP64, PREC_MIXED, MHSError  # noqa: E402
from paper_1307_6720_amd import _lib  # noqa: E402
from paper_1307_6720_amd.solver import Plan, make_opts, solve  # noqa: E402

DEV = "cuda:0"
NAMES = ("P", "Bx", "By", "Bz", "dp", "drho")


def rel(a, b):
    d = np.abs(b).max()
    return float(np.abs(a - b).max() / (d if d > 0 else 1.0))


def field_errors(res, want_P, m):
    want = fields.fields(want_P, m.alpha, m.xi, m.dxi, m.pb, m.rhob, m.mu0, m.g)
    pb = m.pb[:, None, None]
    rb = m.rhob[:, None, None]
    got = [res.P, res.Bx, res.By, res.Bz, res.p, res.rho]
    got = [g.cpu().numpy() for g in got]
    got[4] = got[4] - pb
    got[5] = got[5] - rb
    ref_ = [want_P, want[0], want[1], want[2], want[3] - pb, want[4] - rb]
    return {n: rel(g, w) for n, g, w in zip(NAMES, got, ref_)}


@pytest.fixture(scope="module")
def plans():
    cache = {}

    def get(dims):
        if dims not in cache:
            nx, ny, nz = dims
            cache[dims] = Plan(synth.make_grid(nx, ny, nz), PREC_FP64 | PREC_MIXED, device=DEV)
        return cache[dims]

    yield get
    for p in cache.values():
        p.close()


@pytest.mark.parametrize("dims,cycles", [((33, 33, 33), 1), ((33, 33, 33), 3), ((65, 33, 17), 2),
                                         ((129, 65, 65), 2), ((129, 129, 65), 2), ((33, 33, 5), 3),
                                         ((9, 9, 129), 2), ((5, 5, 257), 2), ((17, 9, 65), 2)])
def test_fixed_cycle_algorithm_parity(plans, dims, cycles):
    """Same V(2,2) method as the oracle's C twin: equal iterates after a fixed
    number of cycles (2D and 3D).  (65, 33, 17) and (129, 129, 65) halve x
    and y alone on their first step; (33, 33, 5) does so on three steps, two
    of them inside the bottom solver; (9, 9, 129), (5, 5, 257) and
    (17, 9, 65) halve z alone on their first steps (inside and outside the
    bottom solver)."""
    nx, ny, nz = dims
    print(f"[solve] fixed cycles {dims} x{cycles}", flush=True)
    w = synth.workload("mhs-129", dims=dims)
    m = w.model
    plan = plans(dims)
    L, kinds = ref.levels3(nx, ny, nz)
    assert plan.levels(3) == L
    shapes = [plan.level_shape(3, l) for l in range(L)]
    got = [ref.STEP_XY if b[0] == a[0] else ref.STEP_Z if b[2] == a[2] else ref.STEP_ALL
           for a, b in zip(shapes, shapes[1:])]
    assert got == kinds
    # 2D: oracle P0 after `cycles` cycles
    P0_ref, st, c2, _ = ref.mg2(w.bz0, rtol=0.0, max_cycles=cycles)
    assert c2 == cycles
    P = torch.zeros((nz, ny, nx), dtype=torch.float64, device=DEV)
    bz = torch.from_numpy(w.bz0).to(DEV)
    info = plan.solve_boundary(bz, P, make_opts(rtol=0.0, max_cycles=cycles), raise_on_error=False)
    assert info.status == _lib.ERR_NO_CONVERGENCE and info.cycles == cycles
    assert rel(P[0].cpu().numpy(), P0_ref) < 1e-12
    # 3D from the oracle's base plane
    ubc = np.zeros((nz, ny, nx))
    ubc[0] = P0_ref
    P3_ref, st, c3, rr = ref.mg3(ubc, m.xi, m.alpha, rtol=0.0, max_cycles=cycles)
    P.copy_(torch.from_numpy(ubc))
    info = plan.solve_interior(m, P, make_opts(rtol=0.0, max_cycles=cycles), raise_on_error=False)
    assert info.status == _lib.ERR_NO_CONVERGENCE and info.cycles == cycles
    assert abs(info.rel_residual - rr) <= 1e-9 * rr
    assert rel(P.cpu().numpy(), P3_ref) < 1e-12


@pytest.mark.parametrize("name,dims,prec,rtol,tol", [
    ("potential-33", (33, 33, 33), PREC_FP64, 1e-12, 1e-10),
    ("potential-33", (33, 33, 33), PREC_MIXED, 1e-10, 1e-8),
    ("mhs-129", (129, 129, 129), PREC_FP64, 1e-12, 1e-10),
    ("mhs-129", (129, 129, 129), PREC_MIXED, 1e-10, 1e-8),
    ("mhs-129", (65, 129, 33), PREC_MIXED, 1e-10, 1e-8),
])
def test_solution_parity(plans, name, dims, prec, rtol, tol):
    print(f"[solve] parity {name} {dims} prec={prec}", flush=True)
    w = synth.workload(name, dims=dims)
    m = w.model
    plan = plans(dims)
    res = solve(plan, torch.from_numpy(w.bz0).to(DEV), m, precision=prec, rtol=rtol)
    torch.cuda.synchronize()
    want_P = exact.solve(w.bz0, dims[2], m.xi, m.alpha)
    errs = field_errors(res, want_P, m)
    print(errs, res.info2d, res.info3d)
    for n, e in errs.items():
        assert e < tol, (n, e)
    if m.xi.max() == 0.0:
        assert errs["dp"] == 0.0 and errs["drho"] == 0.0


@pytest.fixture(scope="module")
def exact257():
    """The exact discrete solution of each run of the 257^3 workload."""
    cache = {}

    def get(run):
        if run not in cache:
            w = synth.workload("mhs-257", run=run)
            cache.clear()  # one run at a time (0.14 GB per solution)
            cache[run] = (w, exact.solve(w.bz0, 257, w.model.xi, w.model.alpha))
        return cache[run]

    return get


@pytest.mark.parametrize("run", range(6))
def test_full_size_257_parity(plans, exact257, run):
    """The headline size, every run the benchmark times (alpha in {0, 0.5,
    1} x a in {0, 0.5}), in its launch configuration and stopping rule
    (rtol 1e-10): every node of P, B, p - p_b, rho - rho_b of both paths
    within 1e-8 of the exact discrete solution, and the mixed path's FP32
    V-cycles (refinement steps times the cycles per step) within one step of
    the FP64 path's V-cycles (a weaker FP32 inner cycle would need more
    steps)."""
    w, want_P = exact257(run)
    m = w.model
    plan = plans((257, 257, 257))
    counts = {}
    for prec in (PREC_FP64, PREC_MIXED):
        print(f"[solve] 257^3 run {run} prec={prec}", flush=True)
        res = solve(plan, torch.from_numpy(w.bz0).to(DEV), m, precision=prec, rtol=1e-10)
        torch.cuda.synchronize()
        errs = field_errors(res, want_P, m)
        print(errs, res.info2d, res.info3d)
        for n, e in errs.items():
            assert e < 1e-8, (prec, n, e)
        counts[prec] = res.info3d["inner_cycles" if prec == PREC_MIXED else "cycles"]
        per_step = res.info3d["inner_cycles"] // max(1, res.info3d["cycles"])
        del res
    assert abs(counts[PREC_MIXED] - counts[PREC_FP64]) <= max(1, per_step), counts


@pytest.mark.parametrize("run", [0, 5])
def test_full_size_257_fp64_to_1e10(plans, exact257, run):
    """The FP64 path at the spec FP64 gate: rtol 1e-12 gives every
    field within 1e-10 of the exact discrete solution at 257^3."""
    print(f"[solve] 257^3 run {run} FP64 rtol 1e-12", flush=True)
    w, want_P = exact257(run)
    m = w.model
    plan = plans((257, 257, 257))
    res = solve(plan, torch.from_numpy(w.bz0).to(DEV), m, precision=PREC_FP64, rtol=1e-12)
    torch.cuda.synchronize()
    errs = field_errors(res, want_P, m)
    print(errs, res.info2d, res.info3d)
    for n, e in errs.items():
        assert e < 1e-10, (n, e)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_mixed_steps_track_fp64_cycles_129(plans, m):
    """At 129^3 (mhs-129) the mixed path with m FP32 V-cycles per refinement
    step needs as many FP32 V-cycles as the FP64 path needs V-cycles, give
    or take one step, at the same rtol: each step's inner cycles contract
    like FP64 cycles, so a weakened FP32 cycle fails this."""
    w = synth.workload("mhs-129")
    plan = plans((129, 129, 129))
    counts = {}
    for prec in (PREC_FP64, PREC_MIXED):
        res = solve(plan, torch.from_numpy(w.bz0).to(DEV), w.model, precision=prec, rtol=1e-10, fields=False,
                    inner_cycles=m)
        counts[prec] = res.info3d["inner_cycles" if prec == PREC_MIXED else "cycles"]
        if prec == PREC_MIXED:
            assert res.info3d["inner_cycles"] == m * res.info3d["cycles"], res.info3d
    assert abs(counts[PREC_MIXED] - counts[PREC_FP64]) <= m, counts


def test_full_size_513_against_exact():
    """The large single equilibrium (513 x 513 x 257, dz = 2 dx, a = 1 so
    that xi(0) = 1, 40 bipoles plus noise), mixed path to rtol 1e-12: every
    node of P, B, p - p_b and rho - rho_b within 1e-8 of the exact discrete
    solution and its field recovery; the first step of the hierarchy halves
    x and y only, and the cycle converges as on an equally spaced grid.
    The rtol is calibrated for this grid: the noise on every node of the
    magnetogram puts energy into the shortest modes, whose error the
    derivatives of B, p and rho amplify; at rtol 1e-10 P is within 7e-10
    but rho - rho_b only within 2.4e-7, at 1e-11 within 3.5e-8, at 1e-12
    within 6e-9 (measured on both paths)."""
    print("[solve] 513x513x257 mixed", flush=True)
    w = synth.workload("mhs-513x513x257")
    m = w.model
    g = w.grid
    plan = Plan(g, PREC_FP64 | PREC_MIXED, device=DEV)
    res = solve(plan, torch.from_numpy(w.bz0).to(DEV), m, precision=PREC_MIXED, rtol=1e-12)
    torch.cuda.synchronize()
    assert res.info2d["status"] == 0 and res.info3d["status"] == 0, (res.info2d, res.info3d)
    assert plan.level_shape(3, 1) == (257, 257, 257)
    assert res.info3d["cycles"] <= 12, res.info3d
    print("[solve] 513x513x257 exact solve and fields on the host", flush=True)
    want_P = exact.solve(w.bz0, g.nz, m.xi, m.alpha, g.lx, g.ly, g.lz)
    want = fields.fields(want_P, m.alpha, m.xi, m.dxi, m.pb, m.rhob, m.mu0, m.g, g.lx, g.ly, g.lz)
    pb = m.pb[:, None, None]
    rb = m.rhob[:, None, None]
    errs = {"P": rel(res.P.cpu().numpy(), want_P)}
    del want_P
    for name, t, wv in zip(("Bx", "By", "Bz"), (res.Bx, res.By, res.Bz), want[:3]):
        errs[name] = rel(t.cpu().numpy(), wv)
    errs["dp"] = rel(res.p.cpu().numpy() - pb, want[3] - pb)
    errs["drho"] = rel(res.rho.cpu().numpy() - rb, want[4] - rb)
    print(errs, res.info2d, res.info3d)
    for n, e in errs.items():
        assert e < 1e-8, (n, e)
    plan.close()


@pytest.mark.parametrize("prec", [PREC_FP64, PREC_MIXED])
def test_graph_replays_equal_eager_launches(plans, prec):
    """A cycle replayed as a captured HIP graph computes what launching its
    kernels one by one does: over several calls in a row (the plan's cached
    graphs replayed, a new P each call, eager solves and other device work
    in between) every result is bitwise the eager one, with the same cycle
    counts."""
    dims = (65, 65, 65)
    w = synth.workload("mhs-129", dims=dims)
    m = w.model
    plan = plans(dims)
    bz = torch.from_numpy(w.bz0).to(DEV)

    def run(graph):
        P = torch.zeros(w.grid.shape, dtype=torch.float64, device=DEV)
        i2 = plan.solve_boundary(bz, P, make_opts(PREC_FP64, 1e-10, graph=graph))
        i3 = plan.solve_interior(m, P, make_opts(prec, 1e-10, graph=graph))
        torch.cuda.synchronize()
        return P, i2, i3

    want, w2, w3 = run(False)
    for k in range(3):
        got, i2, i3 = run(True)
        assert torch.equal(got, want), k
        assert (i2.cycles, i3.cycles, i3.inner_cycles) == (w2.cycles, w3.cycles, w3.inner_cycles)
        x = torch.arange(4096, dtype=torch.float64, device=DEV)
        assert float((x * 2).sum()) == 4095.0 * 4096.0
        again, _, _ = run(False)
        assert torch.equal(again, want)


def test_repeat_is_bitwise_deterministic(plans):
    w = synth.workload("mhs-129", dims=(65, 65, 65))
    plan = plans((65, 65, 65))
    bz = torch.from_numpy(w.bz0).to(DEV)
    a = solve(plan, bz, w.model, precision=PREC_MIXED, rtol=1e-10)
    a = [t.clone() for t in (a.P, a.Bx, a.rho)]
    b = solve(plan, bz, w.model, precision=PREC_MIXED, rtol=1e-10)
    for x, y in zip(a, (b.P, b.Bx, b.rho)):
        assert torch.equal(x, y)


def test_check_every_does_not_change_result(plans):
    """Cycles launched past convergence are no-ops (device-side flag)."""
    w = synth.workload("mhs-129", dims=(65, 65, 65))
    m = w.model
    plan = plans((65, 65, 65))
    bz = torch.from_numpy(w.bz0).to(DEV)
    out = []
    for ce in (1, 3, 50):
        P = torch.zeros((65, 65, 65), dtype=torch.float64, device=DEV)
        plan.solve_boundary(bz, P, make_opts(rtol=1e-10, check_every=ce))
        info = plan.solve_interior(m, P, make_opts(rtol=1e-10, check_every=ce))
        out.append((P.clone(), info.cycles))
    for P, c in out[1:]:
        assert c == out[0][1]
        assert torch.equal(P, out[0][0])


@pytest.mark.parametrize("prec", [PREC_FP64, PREC_MIXED])
def test_repeat_solve_reads_status_once_with_same_result(plans, prec):
    """A plan remembers how many cycles its last converged solve of a kind
    took with the same options: a repeat launches that many plus the
    checking one before its first status read, so it reads the status once,
    and its result is bitwise that of a solve on a fresh plan (batches end
    on a convergence check; launches past convergence exit at once)."""
    w = synth.workload("mhs-129", dims=(65, 65, 65))
    m = w.model
    bz = torch.from_numpy(w.bz0).to(DEV)
    fresh = Plan(w.grid, PREC_FP64 | PREC_MIXED, device=DEV)
    P0 = torch.zeros((65, 65, 65), dtype=torch.float64, device=DEV)
    i2a = fresh.solve_boundary(bz, P0, make_opts(rtol=1e-10))
    i3a = fresh.solve_interior(m, P0, make_opts(prec, rtol=1e-10))
    fresh.close()
    plan = plans((65, 65, 65))
    for rep in range(2):
        P = torch.zeros((65, 65, 65), dtype=torch.float64, device=DEV)
        i2 = plan.solve_boundary(bz, P, make_opts(rtol=1e-10))
        i3 = plan.solve_interior(m, P, make_opts(prec, rtol=1e-10))
        torch.cuda.synchronize()
        assert (i2.cycles, i3.cycles) == (i2a.cycles, i3a.cycles)
        assert torch.equal(P, P0)
    assert i2.host_syncs == 1 and i3.host_syncs == 1, (i2.host_syncs, i3.host_syncs)


def test_mixed_start_from_twin_matches_fresh_plan():
    """After a mixed solve of an odd number of refinement steps, the plan's
    next cold mixed solve starts from P's twin so that the same count ends in
    P without a copy.  Its result is bitwise that of a fresh plan: with the
    predicted count, with an even count (a cap of two steps: the iterate is
    copied back from the twin), and with none (zero magnetogram)."""
    w = synth.workload("mhs-129", dims=(65, 65, 65))
    m = w.model
    bz = torch.from_numpy(w.bz0).to(DEV)
    zero = torch.zeros_like(bz)

    def run(plan, b, rtol, **kw):
        P = torch.zeros((65, 65, 65), dtype=torch.float64, device=DEV)
        plan.solve_boundary(b, P, make_opts(rtol=1e-10))
        info = plan.solve_interior(m, P, make_opts(PREC_MIXED, rtol=rtol, **kw), raise_on_error=False)
        torch.cuda.synchronize()
        return P, info

    def fresh(b, rtol, **kw):
        plan = Plan(w.grid, PREC_FP64 | PREC_MIXED, device=DEV)
        try:
            return run(plan, b, rtol, **kw)
        finally:
            plan.close()

    # a tolerance whose solve takes an odd number of steps
    for rtol in (1e-10, 1e-9, 1e-11, 1e-8, 1e-12):
        want, wi = fresh(bz, rtol)
        assert wi.status == 0, wi.status
        if wi.cycles % 2 == 1 and wi.cycles > 2:
            break
    else:
        pytest.fail("no tolerance gave an odd step count")
    cap, ci = fresh(bz, rtol, max_cycles=2)
    assert ci.status == _lib.ERR_NO_CONVERGENCE and ci.cycles == 2
    none, ni = fresh(zero, rtol)
    assert ni.status == 0 and ni.cycles == 0
    plan = Plan(w.grid, PREC_FP64 | PREC_MIXED, device=DEV)
    try:
        run(plan, bz, rtol)  # records the odd count
        for b, kw, P_want, i_want in ((bz, {}, want, wi), (bz, {"max_cycles": 2}, cap, ci), (zero, {}, none, ni),
                                      (bz, {}, want, wi)):
            P, info = run(plan, b, rtol, **kw)
            assert (info.status, info.cycles) == (i_want.status, i_want.cycles)
            assert torch.equal(P, P_want)
    finally:
        plan.close()


def _three_calls(w, bz, prec, rtol=1e-10, **kw):
    """Boundary, interior and fields as three calls on a fresh plan."""
    plan = Plan(w.grid, PREC_FP64 | PREC_MIXED, device=DEV)
    try:
        P = torch.zeros(w.grid.shape, dtype=torch.float64, device=DEV)
        F = tuple(torch.zeros_like(P) for _ in range(5))
        i2 = plan.solve_boundary(bz, P, make_opts(rtol=1e-10))
        i3 = plan.solve_interior(w.model, P, make_opts(prec, rtol=rtol, **kw), raise_on_error=False)
        if i3.status == 0:
            plan.fields(w.model, P, F)
        torch.cuda.synchronize()
        return P, F, i2, i3
    finally:
        plan.close()


@pytest.mark.parametrize("prec", [PREC_FP64, PREC_MIXED])
def test_equilibrium_call_equals_three_calls(prec):
    """mhs_solve_equilibrium gives bitwise the results of the boundary,
    interior and fields calls made one after the other: on a plan's first
    call, on repeats (where the recovery enqueued behind the converging batch
    is the one that runs), and with no recovery requested."""
    w = synth.workload("mhs-129", dims=(65, 65, 65))
    bz = torch.from_numpy(w.bz0).to(DEV)
    P0, F0, i2a, i3a = _three_calls(w, bz, prec)
    plan = Plan(w.grid, PREC_FP64 | PREC_MIXED, device=DEV)
    try:
        for rep in range(3):
            P = torch.zeros(w.grid.shape, dtype=torch.float64, device=DEV)
            F = tuple(torch.full_like(P, 7.0) for _ in range(5))
            i2, i3 = plan.solve_equilibrium(bz, w.model, P, F, make_opts(rtol=1e-10), make_opts(prec, rtol=1e-10))
            torch.cuda.synchronize()
            assert (i2.cycles, i3.cycles) == (i2a.cycles, i3a.cycles)
            assert torch.equal(P, P0)
            for a, b in zip(F, F0):
                assert torch.equal(a, b)
        P = torch.zeros(w.grid.shape, dtype=torch.float64, device=DEV)
        plan.solve_equilibrium(bz, w.model, P, None, make_opts(rtol=1e-10), make_opts(prec, rtol=1e-10))
        torch.cuda.synchronize()
        assert torch.equal(P, P0)
    finally:
        plan.close()


def test_equilibrium_call_when_the_count_differs_from_the_last():
    """After a mixed solve of an odd number of steps the next one starts
    from P's twin; when its count is even (none for a zero magnetogram, two
    under a cap) the recovery gated on P holding the iterate does not run
    and the call recovers the fields after the copy back (or, capped, stops
    with the copied iterate in P).  A base solve that does not converge ends
    the call with the interior untouched, and the model prepared meanwhile
    is uploaded by the next call."""
    w = synth.workload("mhs-129", dims=(65, 65, 65))
    bz = torch.from_numpy(w.bz0).to(DEV)
    zero = torch.zeros_like(bz)
    for rtol in (1e-10, 1e-9, 1e-11, 1e-8, 1e-12):
        P0, F0, _, i3a = _three_calls(w, bz, PREC_MIXED, rtol)
        if i3a.cycles % 2 == 1 and i3a.cycles > 2:
            break
    else:
        pytest.fail("no tolerance gave an odd step count")
    Pz, Fz, _, iz = _three_calls(w, zero, PREC_MIXED, rtol)
    assert iz.cycles == 0
    Pc, _, _, ic = _three_calls(w, bz, PREC_MIXED, rtol, max_cycles=2)
    assert ic.status == _lib.ERR_NO_CONVERGENCE
    plan = Plan(w.grid, PREC_FP64 | PREC_MIXED, device=DEV)

    def call(b, P, o2=None, **kw):
        F = tuple(torch.full_like(P, 7.0) for _ in range(5))
        i2, i3 = plan.solve_equilibrium(b, w.model, P, F, o2 or make_opts(rtol=1e-10),
                                        make_opts(PREC_MIXED, rtol=rtol, **kw), raise_on_error=False)
        torch.cuda.synchronize()
        return F, i2, i3

    try:
        P = torch.zeros(w.grid.shape, dtype=torch.float64, device=DEV)
        F, _, i3 = call(bz, P)
        assert i3.cycles == i3a.cycles and torch.equal(P, P0)
        P = torch.zeros_like(P)
        F, _, i3 = call(zero, P)
        assert i3.status == 0 and i3.cycles == 0 and torch.equal(P, Pz)
        for a, b in zip(F, Fz):
            assert torch.equal(a, b)
        call(bz, torch.zeros_like(P))  # the odd count again
        P = torch.zeros_like(P)
        _, _, i3 = call(bz, P, max_cycles=2)
        assert i3.status == _lib.ERR_NO_CONVERGENCE and torch.equal(P, Pc)
        # a base solve capped at one cycle: the interior planes keep their values
        fresh = Plan(w.grid, PREC_FP64 | PREC_MIXED, device=DEV)
        try:
            P = torch.full(w.grid.shape, 3.0, dtype=torch.float64, device=DEV)
            F = tuple(torch.full_like(P, 7.0) for _ in range(5))
            i2, _ = fresh.solve_equilibrium(bz, w.model, P, F, make_opts(rtol=1e-10, max_cycles=1),
                                            make_opts(PREC_MIXED, rtol=rtol), raise_on_error=False)
            torch.cuda.synchronize()
            assert i2.status == _lib.ERR_NO_CONVERGENCE
            assert bool((P[1:] == 3.0).all()) and all(bool((t == 7.0).all()) for t in F)
            P = torch.zeros_like(P)
            F = tuple(torch.zeros_like(P) for _ in range(5))
            fresh.solve_equilibrium(bz, w.model, P, F, make_opts(rtol=1e-10), make_opts(PREC_MIXED, rtol=rtol))
            torch.cuda.synchronize()
            assert torch.equal(P, P0)
            for a, b in zip(F, F0):
                assert torch.equal(a, b)
        finally:
            fresh.close()
    finally:
        plan.close()


@pytest.mark.parametrize("faces_given", [False, True])
def test_mixed_cold_start_equals_warm_start_from_zero(faces_given):
    """A cold mixed solve zeroes no interior: its first two refinement steps
    load only the boundary nodes of the start iterate and take its interior
    as zero.  Its result equals that of a warm start from an iterate whose
    interior is zero (which reads every node), whatever the caller's P held
    before; a cold solve that stops at step 0 (zero data) zeroes P's
    interior itself."""
    w = synth.workload("mhs-129", dims=(65, 65, 65))
    bz = torch.from_numpy(w.bz0).to(DEV)
    plan = Plan(w.grid, PREC_FP64 | PREC_MIXED, device=DEV)
    try:
        base = torch.zeros(w.grid.shape, dtype=torch.float64, device=DEV)
        if faces_given:
            gen = torch.Generator(device="cpu").manual_seed(5)
            faces = torch.rand(w.grid.shape, generator=gen, dtype=torch.float64).to(DEV)
            faces[1:-1, 1:-1, 1:-1] = 0.0
            base.copy_(faces)
        plan.solve_boundary(bz, base, make_opts(rtol=1e-10, faces_given=faces_given))
        torch.cuda.synchronize()
        warm = base.clone()
        iw = plan.solve_interior(w.model, warm, make_opts(PREC_MIXED, rtol=1e-10, warm_start=True,
                                                          faces_given=faces_given))
        for rep in range(2):  # the second starts from the twin (odd or even count alike)
            cold = base.clone()
            cold[1:-1, 1:-1, 1:-1] = 5.0  # what the caller's P held: never read
            ic = plan.solve_interior(w.model, cold, make_opts(PREC_MIXED, rtol=1e-10, faces_given=faces_given))
            torch.cuda.synchronize()
            assert ic.cycles == iw.cycles
            assert torch.equal(cold, warm)
        zero = torch.zeros_like(bz)
        P = torch.full(w.grid.shape, 5.0, dtype=torch.float64, device=DEV)
        plan.solve_boundary(zero, P, make_opts(rtol=1e-10))
        i3 = plan.solve_interior(w.model, P, make_opts(PREC_MIXED, rtol=1e-10))
        torch.cuda.synchronize()
        assert i3.cycles == 0
        assert bool((P == 0.0).all())
    finally:
        plan.close()


def test_error_paths(plans):
    w = synth.workload("mhs-129", dims=(33, 33, 33))
    m = w.model
    plan = plans((33, 33, 33))
    P = torch.zeros((33, 33, 33), dtype=torch.float64, device=DEV)
    bad = synth.Model(m.alpha, m.xi.copy(), m.dxi, m.pb, m.rhob)
    bad.xi[5] = 1.0
    with pytest.raises(MHSError) as e:
        plan.solve_interior(bad, P)
    assert e.value.code == _lib.ERR_NOT_ELLIPTIC
    big = synth.Model(7.0, m.xi, m.dxi, m.pb, m.rhob)  # alpha^2 = 49 exceeds pi^2 (1 + 2 min(1 - xi))
    with pytest.raises(MHSError) as e:
        plan.solve_interior(big, P)
    assert e.value.code == _lib.ERR_INDEFINITE
    with pytest.raises(MHSError) as e:
        plan.solve_interior(m, P, make_opts(nu1=0))
    assert e.value.code == _lib.ERR_INVALID_ARG
    bz = torch.from_numpy(w.bz0).to(DEV)
    info = plan.solve_boundary(bz, P, make_opts(rtol=1e-14, max_cycles=2), raise_on_error=False)
    assert info.status == _lib.ERR_NO_CONVERGENCE and info.cycles == 2 and info.rel_residual > 1e-14
    nan_bz = bz.clone()
    nan_bz[5, 5] = float("nan")
    info = plan.solve_boundary(nan_bz, P, make_opts(), raise_on_error=False)
    assert info.status == _lib.ERR_DIVERGED


def test_stage_calls_do_not_disturb_solves(plans):
    """Stage entry points borrow solver scratch buffers; a solve after them
    must be unaffected (regression: an FP32 stage call once left nonzero
    boundary values in the refinement's scratch and broke the next solve)."""
    dims = (65, 65, 65)
    w = synth.workload("mhs-129", dims=dims)
    m = w.model
    plan = plans(dims)
    bz = torch.from_numpy(w.bz0).to(DEV)
    ref_res = solve(plan, bz, m, precision=PREC_MIXED, rtol=1e-10)
    ref_P = ref_res.P.clone()
    u32 = torch.randn(dims[::-1], dtype=torch.float32, device=DEV)
    plan.stage_smooth(m, 3, 0, u32, torch.randn_like(u32), 2, precision=PREC_MIXED)
    u64 = torch.randn(plan.level_shape(3, 1), dtype=torch.float64, device=DEV)
    plan.stage_smooth(m, 3, 1, u64, torch.randn_like(u64), 2)
    plan.stage_residual_norm(m, 3, 1, u64, torch.randn_like(u64))
    again = solve(plan, bz, m, precision=PREC_MIXED, rtol=1e-10)
    assert torch.equal(again.P, ref_P)
    again = solve(plan, bz, m, precision=PREC_FP64, rtol=1e-10)
    assert (again.P - ref_P).abs().max().item() < 1e-8 * ref_P.abs().max().item()


@pytest.mark.parametrize("dims", [(33, 33, 33), (65, 33, 17)])
def test_given_faces_fixed_cycles_and_exact_trilinear(plans, dims):
    """Dirichlet data given on every face (opts.faces = MHS_FACES_GIVEN):
    the same iterates as the oracle's twin after a fixed number of cycles
    (2D with given edges, then 3D with given side and top faces), and a
    trilinear P with alpha = 0 is reproduced by both paths (its second
    differences vanish, so it solves (8) for any xi)."""
    nx, ny, nz = dims
    print(f"[solve] given faces {dims}", flush=True)
    w = synth.workload("mhs-129", dims=dims)
    m = w.model
    plan = plans(dims)
    rng = np.random.default_rng(sum(dims))
    faces = rng.normal(size=(nz, ny, nx))
    faces[1:-1, 1:-1, 1:-1] = 0.0
    # 2D: edges of plane 0 given
    e2 = faces[0].copy()
    e2[1:-1, 1:-1] = 0.0
    P0_ref, _, c2, _ = ref.mg2(w.bz0, rtol=0.0, max_cycles=2, P0=e2, keep_edges=True)
    P = torch.from_numpy(faces.copy()).to(DEV)
    P[0, 1:-1, 1:-1] = 7.0  # interior of plane 0 is not an input
    bz = torch.from_numpy(w.bz0).to(DEV)
    info = plan.solve_boundary(bz, P, make_opts(rtol=0.0, max_cycles=2, faces_given=True), raise_on_error=False)
    assert info.cycles == 2
    assert rel(P[0].cpu().numpy(), P0_ref) < 1e-12
    # 3D: side and top faces given, base from the 2D solve
    ubc = faces.copy()
    ubc[0] = P0_ref
    P3_ref, _, _, rr = ref.mg3(ubc, m.xi, m.alpha, rtol=0.0, max_cycles=2)
    P.copy_(torch.from_numpy(ubc))
    info = plan.solve_interior(m, P, make_opts(rtol=0.0, max_cycles=2, faces_given=True), raise_on_error=False)
    assert info.cycles == 2 and abs(info.rel_residual - rr) <= 1e-9 * rr
    assert rel(P.cpu().numpy(), P3_ref) < 1e-12
    # a trilinear P (alpha = 0) from its faces, both precisions
    z, y, x = np.meshgrid(np.linspace(0, 1, nz), np.linspace(0, 1, ny), np.linspace(0, 1, nx), indexing="ij")
    u = 1.0 + x - 2 * y + 0.5 * z + x * y - y * z + 3 * x * z + x * y * z
    m0 = synth.Model(0.0, m.xi, m.dxi, m.pb, m.rhob)
    for prec, tol in ((PREC_FP64, 1e-10), (PREC_MIXED, 1e-8)):
        bc = u.copy()
        bc[1:-1, 1:-1, 1:-1] = 0.0
        P.copy_(torch.from_numpy(bc))
        plan.solve_interior(m0, P, make_opts(prec, rtol=1e-12 if prec == PREC_FP64 else 1e-10, faces_given=True))
        assert rel(P.cpu().numpy(), u) < tol, prec
    # the default still zeroes the faces
    P.copy_(torch.from_numpy(ubc))
    plan.solve_interior(m, P, make_opts(rtol=0.0, max_cycles=1), raise_on_error=False)
    Ph = P.cpu().numpy()
    assert np.all(Ph[-1] == 0) and np.all(Ph[:, 0] == 0) and np.all(Ph[:, :, -1] == 0)


def test_zero_magnetogram_gives_the_background():
    """Bz0 = 0: r0 = 0, so both solves stop at once with P = 0; then B = 0,
    p = p_b and rho = rho_b on every node."""
    print("[solve] zero magnetogram", flush=True)
    w = synth.workload("mhs-129", dims=(33, 33, 33))
    m = w.model
    plan = Plan(w.grid, PREC_FP64 | PREC_MIXED, device=DEV)
    for prec in (PREC_FP64, PREC_MIXED):
        res = solve(plan, torch.zeros((33, 33), dtype=torch.float64, device=DEV), m, precision=prec)
        assert res.info2d["status"] == 0 and res.info3d["status"] == 0
        assert res.info2d["cycles"] == 0 and res.info3d["cycles"] == 0
        assert torch.count_nonzero(res.P) == 0
        for B in (res.Bx, res.By, res.Bz):
            assert torch.count_nonzero(B) == 0
        assert np.array_equal(res.p.cpu().numpy(), np.broadcast_to(m.pb[:, None, None], (33, 33, 33)))
        assert np.array_equal(res.rho.cpu().numpy(), np.broadcast_to(m.rhob[:, None, None], (33, 33, 33)))
    plan.close()


@pytest.mark.parametrize("dims,lengths", [((5, 5, 5), (1.0, 1.0, 1.0)), ((5, 5, 257), (1.0, 1.0, 64.0)),
                                          ((257, 5, 9), (1.0, 1.0 / 64, 1.0 / 32)), ((9, 129, 5), (0.3, 2.0, 0.05))])
def test_extreme_shapes_match_exact(dims, lengths):
    """The smallest grid (two levels) and long thin boxes (an axis of 5
    nodes beside one of 257, spacings within a factor 3 of each other; the
    hierarchy stops when an axis to be halved has 3 nodes and the coarsest
    grid holds up to a few hundred unknowns): both paths against the exact
    discrete solution."""
    nx, ny, nz = dims
    print(f"[solve] extreme shape {dims} {lengths}", flush=True)
    grid = synth.make_grid(nx, ny, nz, *lengths)
    rng = np.random.default_rng(nx + ny + nz)
    bz0 = np.zeros((ny, nx))
    bz0[1:-1, 1:-1] = rng.normal(size=(ny - 2, nx - 2))
    m = synth.make_model(grid, 0.3, 0.5, 0.3 * lengths[2])
    plan = Plan(grid, PREC_FP64 | PREC_MIXED, device=DEV)
    want = exact.solve(bz0, nz, m.xi, m.alpha, *lengths)
    for prec, rtol, tol in ((PREC_FP64, 1e-12, 1e-10), (PREC_MIXED, 1e-10, 1e-8)):
        res = solve(plan, torch.from_numpy(bz0).to(DEV), m, precision=prec, rtol=rtol, max_cycles=200)
        assert res.info2d["status"] == 0 and res.info3d["status"] == 0, (res.info2d, res.info3d)
        assert rel(res.P.cpu().numpy(), want) < tol, (prec, rel(res.P.cpu().numpy(), want))
    plan.close()


@pytest.mark.parametrize("dims", [(5, 5, 257), (9, 9, 257), (17, 17, 257)])
def test_dz_much_below_dx_converges(dims):
    """dz = dx / 64 .. dx / 8 on the unit cube: the first steps halve z
    alone until the spacing is equal, and both paths converge in about as
    many cycles as on an equally spaced grid, to the exact solution (with
    every axis halved at each step the 5 x 5 x 257 solve stalls: its
    contraction is close to 1)."""
    nx, ny, nz = dims
    print(f"[solve] dz << dx {dims}", flush=True)
    grid = synth.make_grid(nx, ny, nz)
    m = synth.make_model(grid, 0.3, 0.5, 0.3)
    bz0 = np.zeros((ny, nx))
    bz0[1:-1, 1:-1] = np.random.default_rng(3).normal(size=(ny - 2, nx - 2))
    want = exact.solve(bz0, nz, m.xi, m.alpha)
    plan = Plan(grid, PREC_FP64 | PREC_MIXED, device=DEV)
    assert plan.level_shape(3, 1) == ((nz - 1) // 2 + 1, ny, nx)
    for prec, rtol, tol in ((PREC_FP64, 1e-12, 1e-10), (PREC_MIXED, 1e-10, 1e-8)):
        res = solve(plan, torch.from_numpy(bz0).to(DEV), m, precision=prec, rtol=rtol, max_cycles=40)
        assert res.info3d["status"] == 0 and res.info3d["cycles"] <= 14, res.info3d
        assert rel(res.P.cpu().numpy(), want) < tol
    plan.close()
