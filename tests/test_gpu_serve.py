"""Serving on the GPU: every request gives the same result alone (the
single-request entry points) and in the mix (merged batch launches), bit
for bit, whatever else is in the batch; failures stay with their request;
results also match the exact discrete solution (oracle) to the stated
tolerance."""

import numpy as np
import pytest

import synth
from oracle import exact, fields

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1307_6720_amd import PREC_FP64, PREC_MIXED, _lib  # noqa: E402
from paper_1307_6720_amd.serve import Batch, DeviceBackend, Request, Server  # noqa: E402
from paper_1307_6720_amd.solver import Plan, make_opts, solve  # noqa: E402

DEV = "cuda:0"

# (dims (nx, ny, nz), lengths, alpha, a, precision, rtol)
CASES = [
    ((33, 33, 33), (1.0, 1.0, 1.0), 0.0, 0.0, PREC_FP64, 1e-12),
    ((65, 65, 65), (1.0, 1.0, 1.0), 0.5, 0.5, PREC_MIXED, 1e-10),
    ((65, 33, 17), (1.0, 0.6, 0.4), 0.3, 0.2, PREC_FP64, 1e-10),
    ((129, 129, 65), (1.0, 1.0, 0.5), 1.0, 0.5, PREC_MIXED, 1e-10),
    ((33, 65, 129), (1.0, 1.3, 0.8), 0.7, 0.6, PREC_MIXED, 1e-10),
    ((65, 65, 65), (1.0, 1.0, 1.0), 0.9, 0.3, PREC_FP64, 1e-10),
    ((129, 129, 129), (1.0, 1.0, 1.0), 0.5, 0.5, PREC_MIXED, 1e-10),
    # steps that halve z alone (dz = dx / 8), and x and y alone (dz = 2 dx)
    ((17, 17, 129), (1.0, 1.0, 1.0), 0.4, 0.5, PREC_MIXED, 1e-10),
    ((65, 65, 33), (1.0, 1.0, 1.0), 0.2, 0.4, PREC_FP64, 1e-10),
]


def make_request(i, case, seed=500):
    dims, lengths, alpha, a, prec, rtol = case
    nx, ny, nz = dims
    grid = synth.make_grid(nx, ny, nz, *lengths)
    rng = np.random.default_rng(seed + i)
    bz0 = synth.bipolar_magnetogram(nx, ny, grid.lx, grid.ly, 3 + i % 4, rng, sigma=None)
    model = synth.make_model(grid, alpha, a, 0.2 * lengths[2])
    return Request(id=i, dims=dims, model=model, bz0=bz0, precision=prec, rtol=rtol, lengths=lengths)


def alone(req):
    nx, ny, nz = req.dims
    plan = Plan(synth.make_grid(nx, ny, nz, *req.lengths), PREC_FP64 | PREC_MIXED, device=DEV)
    res = solve(plan, torch.from_numpy(req.bz0).to(DEV), req.model, precision=req.precision, rtol=req.rtol)
    torch.cuda.synchronize()
    out = [t.clone() for t in (res.P, res.Bx, res.By, res.Bz, res.p, res.rho)]
    plan.close()
    return out, res.info2d, res.info3d


@pytest.fixture(scope="module")
def alone_results():
    reqs = [make_request(i, c) for i, c in enumerate(CASES)]
    print("[serve] alone solves", flush=True)
    return reqs, [alone(r) for r in reqs]


def serve(reqs, max_slots, budget=64 << 30, gaps=None):
    got = {}

    def keep(req, res):
        got[req.id] = [t.clone() for t in (res.P, *res.F)]

    be = DeviceBackend(max_slots=max_slots, device=DEV)
    srv = Server(be, budget, on_finish=keep)
    for k, r in enumerate(reqs):
        r.arrival = 0.0 if gaps is None else gaps * k
        r.status = r.finished = r.admitted = None
    done, stats = srv.run(reqs)
    torch.cuda.synchronize()
    be.close()
    return {r.id: r for r in done}, got, stats


@pytest.mark.parametrize("max_slots,gaps", [(8, None), (3, 2e-4), (1, None)])
def test_same_result_alone_and_in_the_mix(alone_results, max_slots, gaps):
    reqs, ref = alone_results
    print(f"[serve] mix max_slots={max_slots} gaps={gaps}", flush=True)
    done, got, stats = serve(reqs, max_slots, gaps=gaps)
    assert stats["ok"] == len(reqs)
    assert stats["peak_active"] <= max_slots
    for r in reqs:
        want, i2, i3 = ref[r.id]
        d = done[r.id]
        assert d.status == 0
        assert d.info2d["cycles"] == i2["cycles"] and d.info3d["cycles"] == i3["cycles"], r.id
        for name, a, b in zip(("P", "Bx", "By", "Bz", "p", "rho"), got[r.id], want):
            assert torch.equal(a, b), (r.id, name, (a - b).abs().max().item())


def test_failures_stay_with_their_request(alone_results):
    reqs, ref = alone_results
    keep = [make_request(i, c) for i, c in enumerate(CASES[:3])]
    nan_req = make_request(10, CASES[1])
    nan_req.bz0 = nan_req.bz0.copy()
    nan_req.bz0[7, 9] = np.nan
    bad = make_request(11, CASES[0])
    xi = bad.model.xi.copy()
    xi[4] = 1.0
    bad.model = synth.Model(bad.model.alpha, xi, bad.model.dxi, bad.model.pb, bad.model.rhob)
    capped = make_request(12, CASES[2])
    capped.rtol = 0.0  # never converges: stops at max_cycles
    print("[serve] failures", flush=True)
    done, got, stats = serve(keep + [nan_req, bad, capped], max_slots=4)
    assert done[10].status == _lib.ERR_DIVERGED
    assert done[11].status == _lib.ERR_NOT_ELLIPTIC
    assert done[12].status == _lib.ERR_NO_CONVERGENCE and done[12].info2d["cycles"] == 100
    for r in keep:
        want, _, _ = ref[r.id]
        for a, b in zip(got[r.id], want):
            assert torch.equal(a, b)


def test_batch_result_matches_exact_solution(alone_results):
    reqs, _ = alone_results
    r = make_request(1, CASES[1])
    done, got, _ = serve([r], max_slots=2)
    m = r.model
    nx, ny, nz = r.dims
    lx, ly, lz = r.lengths
    P_ex = exact.solve(r.bz0, nz, m.xi, m.alpha, lx, ly, lz)
    want = fields.fields(P_ex, m.alpha, m.xi, m.dxi, m.pb, m.rhob, m.mu0, m.g, lx, ly, lz)
    P, Bx, By, Bz, p, rho = [t.cpu().numpy() for t in got[1]]
    pb, rb = m.pb[:, None, None], m.rhob[:, None, None]

    def rel(a, b):
        return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))

    assert rel(P, P_ex) < 1e-8
    for a, b in ((Bx, want[0]), (By, want[1]), (Bz, want[2]), (p - pb, want[3] - pb), (rho - rb, want[4] - rb)):
        assert rel(a, b) < 1e-8


def test_batch_abi_direct():
    """mhs_batch_* without the server: slots, polling, release and reuse."""
    reqs = [make_request(i, CASES[i]) for i in (0, 2)]
    b = Batch(2, DEV)
    plans, outs, slots = [], [], []
    for r in reqs:
        nx, ny, nz = r.dims
        plan = Plan(synth.make_grid(nx, ny, nz, *r.lengths), PREC_FP64 | PREC_MIXED, device=DEV)
        P = torch.zeros((nz, ny, nx), dtype=torch.float64, device=DEV)
        F = tuple(torch.empty_like(P) for _ in range(5))
        bz = torch.from_numpy(r.bz0).to(DEV)
        slots.append(b.admit(plan, r.model, bz, P, F, make_opts(r.precision, r.rtol)))
        plans.append(plan)
        outs.append((bz, P, F))
    # a third request does not fit two slots; a plan cannot be admitted twice
    with pytest.raises(_lib.MHSError) as e:
        b.admit(plans[0], reqs[0].model, outs[0][0], outs[0][1], outs[0][2], make_opts())
    assert e.value.code in (_lib.ERR_BUDGET, _lib.ERR_INVALID_ARG)
    ticks = 0
    while True:
        n = b.step()
        ticks += 1
        if n == 0:
            break
        assert ticks < 500
    for s in slots:
        done, i2, i3 = b.poll(s)
        assert done and i2["status"] == 0 and i3["status"] == 0
        assert ticks >= i2["cycles"] + i3["cycles"]
    # release and reuse a slot with the other plan
    b.release(slots[0])
    r = reqs[0]
    P2 = torch.zeros_like(outs[0][1])
    F2 = tuple(torch.empty_like(P2) for _ in range(5))
    s2 = b.admit(plans[0], r.model, outs[0][0], P2, F2, make_opts(r.precision, r.rtol))
    while b.step():
        pass
    done, _, _ = b.poll(s2)
    assert done
    assert torch.equal(P2, outs[0][1])
    b.close()
    for p in plans:
        p.close()


def test_batch_profile_counts_merged_launches(alone_results):
    """mhs_batch_profile_*: merged launches are timed per class, their
    compulsory bytes add up over the requests whose items ran, and timing
    does not change any result."""
    from paper_1307_6720_amd import _lib as L

    reqs, ref = alone_results
    pick = [make_request(i, CASES[i]) for i in (1, 3)]  # two mixed-precision requests
    b = Batch(2, DEV)
    b.profile(True, ["smooth_l0", "refine"])
    plans, outs = [], []
    for r in pick:
        nx, ny, nz = r.dims
        plan = Plan(synth.make_grid(nx, ny, nz, *r.lengths), PREC_FP64 | PREC_MIXED, device=DEV)
        P = torch.zeros((nz, ny, nx), dtype=torch.float64, device=DEV)
        F = tuple(torch.empty_like(P) for _ in range(5))
        b.admit(plan, r.model, torch.from_numpy(r.bz0).to(DEV), P, F, make_opts(r.precision, r.rtol))
        plans.append(plan)
        outs.append((P, F))
    while b.step():
        pass
    prof = b.profile_read(reset=True)
    b.close()
    ms, n, by = prof["smooth_l0"]
    assert n > 0 and ms > 0
    # every level-0 FP32 sweep of a request moves 8, 12 or 12.5 B per node:
    # the class total is a combination of those, bounded by the extremes
    nodes = sum(np.prod(r.dims) for r in pick)
    assert by > 0 and by <= n * 12.5 * 4 * nodes
    assert prof["refine"][1] > 0
    for r, (P, F), plan in zip(pick, outs, plans):
        want = ref[r.id][0]
        for a, w in zip((P, *F), want):
            assert torch.equal(a, w)
        plan.close()


def test_release_before_first_tick_keeps_plan_consistent(alone_results):
    """Admission only prepares the model tables; a slot released before its
    first tick never uploads them, and the plan must not believe it holds
    that model: a later single-request solve with the same model is right."""
    reqs, ref = alone_results
    r = make_request(2, CASES[2])
    nx, ny, nz = r.dims
    plan = Plan(synth.make_grid(nx, ny, nz, *r.lengths), PREC_FP64 | PREC_MIXED, device=DEV)
    b = Batch(1, DEV)
    P = torch.zeros((nz, ny, nx), dtype=torch.float64, device=DEV)
    F = tuple(torch.empty_like(P) for _ in range(5))
    bz = torch.from_numpy(r.bz0).to(DEV)
    s = b.admit(plan, r.model, bz, P, F, make_opts(r.precision, r.rtol))
    b.release(s)  # no tick ran: the tables were never copied
    b.close()
    res = solve(plan, bz, r.model, precision=r.precision, rtol=r.rtol)
    torch.cuda.synchronize()
    want = ref[r.id][0]
    for a, w in zip((res.P, res.Bx, res.By, res.Bz, res.p, res.rho), want):
        assert torch.equal(a, w)
    plan.close()


def test_batch_with_given_faces_equals_single_solve():
    """A request whose faces are given (opts.faces = MHS_FACES_GIVEN) in a
    batch beside a default request: the batch keeps its faces and gives
    bitwise the result of the single-request calls."""
    reqs = [make_request(i, CASES[i]) for i in (0, 1)]
    b = Batch(2, DEV)
    plans, outs, slots, singles = [], [], [], []
    rng = np.random.default_rng(5)
    print("[serve] given faces in a batch", flush=True)
    for q, r in enumerate(reqs):
        nx, ny, nz = r.dims
        plan = Plan(synth.make_grid(nx, ny, nz, *r.lengths), PREC_FP64 | PREC_MIXED, device=DEV)
        faces = np.zeros((nz, ny, nx))
        if q == 0:
            faces = rng.normal(size=(nz, ny, nx))
            faces[1:-1, 1:-1, 1:-1] = 0.0
        o = make_opts(r.precision, r.rtol, faces_given=(q == 0))
        bz = torch.from_numpy(r.bz0).to(DEV)
        # single-request calls first
        Ps = torch.from_numpy(faces.copy()).to(DEV)
        plan.solve_boundary(bz, Ps, o)
        plan.solve_interior(r.model, Ps, o)
        Fs = tuple(torch.empty_like(Ps) for _ in range(5))
        plan.fields(r.model, Ps, Fs)
        singles.append((Ps, Fs))
        P = torch.from_numpy(faces.copy()).to(DEV)
        F = tuple(torch.empty_like(P) for _ in range(5))
        slots.append(b.admit(plan, r.model, bz, P, F, o))
        plans.append(plan)
        outs.append((P, F))
    while b.step():
        pass
    for s, (P, F), (Ps, Fs) in zip(slots, outs, singles):
        done, i2, i3 = b.poll(s)
        assert done and i2["status"] == 0 and i3["status"] == 0
        assert torch.equal(P, Ps)
        assert all(torch.equal(a, c) for a, c in zip(F, Fs))
    P0 = outs[0][0].cpu().numpy()
    assert np.abs(P0[-1]).max() > 0 and np.abs(P0[:, 0]).max() > 0  # faces kept
    b.close()
    for p in plans:
        p.close()


def test_merged_257_batch_equals_single_solves():
    """The headline configuration: 257^3 requests (three runs of the
    benchmark's workload, both precisions) merged into one batch give bit
    for bit the single-request results.  Merged launches chunk the z-march
    of levels >= 1 differently from a single request; those levels carry no
    reductions, so nothing may change."""
    runs = [(1, PREC_MIXED), (2, PREC_FP64), (4, PREC_MIXED)]
    works = [synth.workload("mhs-257", run=r) for r, _ in runs]
    plans = [Plan(w.grid, PREC_FP64 | PREC_MIXED, device=DEV) for w in works]
    singles = []
    for (r, prec), w, plan in zip(runs, works, plans):
        print(f"[serve] 257^3 run {r} alone", flush=True)
        res = solve(plan, torch.from_numpy(w.bz0).to(DEV), w.model, precision=prec, rtol=1e-10)
        torch.cuda.synchronize()
        singles.append(([t.clone() for t in (res.P, res.Bx, res.By, res.Bz, res.p, res.rho)],
                        res.info2d["cycles"], res.info3d["cycles"]))
        del res
    print("[serve] 257^3 runs merged", flush=True)
    b = Batch(len(runs), DEV)
    outs, slots = [], []
    for (r, prec), w, plan in zip(runs, works, plans):
        P = torch.zeros(w.grid.shape, dtype=torch.float64, device=DEV)
        F = tuple(torch.empty_like(P) for _ in range(5))
        bz = torch.from_numpy(w.bz0).to(DEV)
        slots.append(b.admit(plan, w.model, bz, P, F, make_opts(prec, 1e-10)))
        outs.append((bz, P, F))
    while b.step():
        pass
    torch.cuda.synchronize()
    for s, (bz, P, F), (want, c2, c3) in zip(slots, outs, singles):
        done, i2, i3 = b.poll(s)
        assert done and i2["status"] == 0 and i3["status"] == 0
        assert (i2["cycles"], i3["cycles"]) == (c2, c3)
        for name, a, w_ in zip(("P", "Bx", "By", "Bz", "p", "rho"), (P, *F), want):
            assert torch.equal(a, w_), (name, (a - w_).abs().max().item())
    b.close()
    for p in plans:
        p.close()


def test_batch_refuses_admission_over_its_budget():
    """mhs_batch_create's HBM budget: a request whose footprint
    (mhs_request_bytes) would take the batch over it is refused with
    MHS_ERR_BUDGET; after a release it fits again."""
    from paper_1307_6720_amd.solver import request_bytes

    reqs = [make_request(i, CASES[1]) for i in range(2)]  # 65^3, mixed
    nx, ny, nz = reqs[0].dims
    grid = synth.make_grid(nx, ny, nz)
    one = request_bytes(grid)
    b = Batch(4, DEV, hbm_budget=one + one // 2)
    plans, outs = [], []
    for r in reqs:
        plan = Plan(grid, PREC_FP64 | PREC_MIXED, device=DEV)
        P = torch.zeros((nz, ny, nx), dtype=torch.float64, device=DEV)
        F = tuple(torch.empty_like(P) for _ in range(5))
        plans.append(plan)
        outs.append((torch.from_numpy(r.bz0).to(DEV), P, F))
    s0 = b.admit(plans[0], reqs[0].model, *outs[0], make_opts(PREC_MIXED, 1e-10))
    assert b.bytes_in_use() == one
    with pytest.raises(_lib.MHSError) as e:
        b.admit(plans[1], reqs[1].model, *outs[1], make_opts(PREC_MIXED, 1e-10))
    assert e.value.code == _lib.ERR_BUDGET
    while b.step():
        pass
    assert b.poll(s0)[0]
    b.release(s0)
    assert b.bytes_in_use() == 0
    s1 = b.admit(plans[1], reqs[1].model, *outs[1], make_opts(PREC_MIXED, 1e-10))
    while b.step():
        pass
    assert b.poll(s1)[0]
    b.close()
    for p in plans:
        p.close()


def test_budget_bound_serving_queues_evicts_and_matches_alone():
    """A serving run on the device whose HBM budget binds: 65^3 and 257^3
    requests under a budget that holds one 257^3 request, or several small
    ones, but not both.  The 257^3 request waits until the small ones have
    finished and their idle residents are evicted; the small request behind
    it waits for the 257^3 one and evicts it in turn.  The in-flight
    footprint never exceeds the budget, and every result is bit for bit its
    single-request result."""
    from paper_1307_6720_amd.solver import request_bytes

    small = (65, 65, 65)
    big = (257, 257, 257)
    one = (1.0, 1.0, 1.0)
    cases = [(small, one, 0.3, 0.2, PREC_MIXED, 1e-10),
             (small, one, 0.8, 0.6, PREC_FP64, 1e-10),
             (small, one, 0.5, 0.5, PREC_MIXED, 1e-10),
             (big, one, 0.5, 0.5, PREC_MIXED, 1e-10),
             (small, one, 0.1, 0.9, PREC_FP64, 1e-10)]
    reqs = [make_request(i, c, seed=900) for i, c in enumerate(cases)]
    fp_big = request_bytes(synth.make_grid(*big))
    fp_small = request_bytes(synth.make_grid(*small))
    budget = fp_big + fp_small // 2
    print(f"[serve] budget {budget / 2**30:.3f} GiB (257^3 request {fp_big / 2**30:.3f} GiB)", flush=True)
    want = {r.id: alone(r) for r in reqs}
    got = {}
    in_use = []
    freed = []

    def keep(req, res):
        got[req.id] = [t.clone() for t in (res.P, *res.F)]

    be = DeviceBackend(max_slots=4, device=DEV, hbm_budget=budget)
    srv = Server(be, budget, on_finish=keep)
    orig_step, orig_free = be.step, be.free

    def step():
        in_use.append(be.batch.bytes_in_use())
        return orig_step()

    def free(res):
        freed.append(res.key[0])
        return orig_free(res)

    be.step, be.free = step, free
    for r in reqs:
        r.arrival = 0.0
    done, stats = srv.run(reqs)
    torch.cuda.synchronize()
    be.close()
    assert stats["ok"] == len(reqs)
    assert stats["peak_resident_bytes"] <= budget and max(in_use) <= budget
    d = {x.id: x for x in done}
    small_done = max(d[i].finished for i in (0, 1, 2))
    assert d[3].admitted >= small_done  # the 257^3 request waited for memory
    assert d[4].admitted >= d[3].finished  # and the last small one for it
    assert freed.count(small) >= 1 and freed.count(big) >= 1  # idle residents were evicted
    for r in reqs:
        w, i2, i3 = want[r.id]
        assert d[r.id].status == 0 and d[r.id].info3d["cycles"] == i3["cycles"]
        for name, a, b_ in zip(("P", "Bx", "By", "Bz", "p", "rho"), got[r.id], w):
            assert torch.equal(a, b_), (r.id, name)
