"""Field-line tracing: the oracle pinned against exact interpolation,
straight lines of a uniform field, the helices of a linear field (fourth
order in the step), reversal symmetry and the spine and fan of a linear
null (CPU); the GPU kernel against the oracle line by line (GPU)."""

import numpy as np
import pytest

import synth
from oracle import fieldlines as ofl


def grid_coords(shape, lengths):
    nz, ny, nx = shape
    lx, ly, lz = lengths
    return np.meshgrid(np.linspace(0, lz, nz), np.linspace(0, ly, ny), np.linspace(0, lx, nx), indexing="ij")


def trilinear(c, x, y, z):
    return (c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * y * z + c[6] * x * z
            + c[7] * x * y * z)


def test_interpolation_exact_on_trilinear_fields():
    """Trilinear interpolation reproduces a field that is trilinear in
    (x, y, z) everywhere, and the node values at nodes (to rounding: a node's
coordinate over the spacing may fall an ulp short of its index); points outside the
    box take the value at the clamped point."""
    shape, lengths = (9, 17, 5), (1.0, 0.7, 1.6)
    z, y, x = grid_coords(shape, lengths)
    c = np.random.default_rng(1).normal(size=8)
    F = trilinear(c, x, y, z)
    rng = np.random.default_rng(2)
    pos = rng.uniform(0, 1, size=(500, 3)) * np.array(lengths)
    got = ofl.sample(F, pos, lengths)
    want = trilinear(c, pos[:, 0], pos[:, 1], pos[:, 2])
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()
    nodes = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    assert np.abs(ofl.sample(F, nodes, lengths) - F.ravel()).max() < 1e-15 * np.abs(F).max() * 8
    far = np.array([[-0.5, 0.3, 0.4], [0.2, 9.0, -1.0]])
    clamped = np.array([[0.0, 0.3, 0.4], [0.2, 0.7, 0.0]])
    assert np.array_equal(ofl.sample(F, far, lengths), ofl.sample(F, clamped, lengths))


def test_uniform_field_gives_straight_lines():
    shape, lengths = (9, 9, 9), (1.0, 1.0, 1.0)
    B = [np.full(shape, v) for v in (1.0, 2.0, 2.0)]
    u = np.array([1.0, 2.0, 2.0]) / 3.0
    seeds = np.array([[0.1, 0.05, 0.203], [0.5, 0.5, 0.5013]])  # no step lands on a face
    ds = 0.01
    pts, count, status = ofl.trace(*B, seeds, ds, 500, 0.0, lengths)
    for l, x0 in enumerate(seeds):
        # the last step that stays in the box: y or z reaches 1 first
        nmax = int(np.floor(min((1.0 - x0[a]) / (ds * u[a]) for a in range(3)) + 1e-9))
        assert count[l] == nmax + 1 and status[l] == ofl.EXIT
        n = np.arange(count[l])[:, None]
        want = x0 + n * ds * u
        assert np.abs(pts[: count[l], l] - want).max() < 1e-14


def helix_case(n, x0=0.5, y0=0.45, c=0.6):
    shape, lengths = (n, n, n), (1.0, 1.0, 1.0)
    z, y, x = grid_coords(shape, lengths)
    return (-(y - y0), x - x0, np.full(shape, c)), lengths


def test_linear_field_gives_helices_to_fourth_order():
    """B = (-(y - y0), x - x0, c) is reproduced exactly by the interpolation;
    its lines are helices of radius r about (x0, y0) with |B| = sqrt(r^2 +
    c^2) constant, turning at 1/|B| per unit arc length and rising at
    c/|B|.  RK4's error after a fixed arc length falls as ds^4."""
    x0, y0, c = 0.5, 0.45, 0.3
    B, lengths = helix_case(9, x0, y0, c)
    seed = np.array([[0.7, 0.45, 0.1]])
    r, th0 = 0.2, 0.0
    bn = np.hypot(r, c)
    S = 0.8
    errs = []
    for ds in (0.08, 0.04, 0.02):
        steps = int(round(S / ds))
        pts, count, status = ofl.trace(*B, seed, ds, steps, 0.0, lengths)
        assert count[0] == steps + 1 and status[0] == ofl.MAXSTEPS
        s = steps * ds
        want = np.array([x0 + r * np.cos(th0 + s / bn), y0 + r * np.sin(th0 + s / bn), 0.1 + c * s / bn])
        errs.append(np.abs(pts[steps, 0] - want).max())
    assert errs[0] / errs[1] > 12 and errs[1] / errs[2] > 12, errs
    assert errs[-1] < 5e-8


def test_negative_step_equals_reversed_field():
    B, lengths = helix_case(9)
    rng = np.random.default_rng(3)
    seeds = rng.uniform(0.2, 0.8, size=(20, 3))
    a = ofl.trace(*B, seeds, -0.03, 60, 0.0, lengths)
    b = ofl.trace(*[-F for F in B], seeds, 0.03, 60, 0.0, lengths)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_linear_null_spine_and_fan():
    """B = (x - x0, y - y0, -2 (z - z0)) (divergence-free, a null at (x0, y0,
    z0) on a node): a seed on the spine runs down the spine, x and y fixed
    exactly, and stops at the null; a seed in the fan plane runs outward in
    that plane and leaves the box."""
    n = 17
    shape, lengths = (n, n, n), (1.0, 1.0, 1.0)
    z, y, x = grid_coords(shape, lengths)
    x0, y0, z0 = 0.5, 0.5, 0.25
    B = (x - x0, y - y0, -2.0 * (z - z0))
    seeds = np.array([[x0, y0, 0.6], [0.7, 0.6, z0]])
    bmin = 1e-3
    pts, count, status = ofl.trace(*B, seeds, 0.01, 1000, bmin, lengths)
    sp = pts[: count[0], 0]
    assert status[0] == ofl.NULL
    assert np.all(sp[:, 0] == x0) and np.all(sp[:, 1] == y0)
    assert np.all(np.diff(sp[:, 2]) < 0) and abs(sp[-1, 2] - z0) < 0.01 + bmin
    fan = pts[: count[1], 1]
    assert status[1] == ofl.EXIT
    assert np.all(fan[:, 2] == z0)
    # radial: the direction from the null stays that of the seed
    d = fan[:, :2] - np.array([x0, y0])
    assert np.abs(d[:, 0] * 0.1 - d[:, 1] * 0.2).max() < 1e-13


def test_exact_null_at_a_node_ends_the_line():
    """|B| = 0 exactly (a null on a node, bmin = 0): the line that reaches
    it ends there with status NULL, and no stage produces NaN."""
    n = 9
    shape, lengths = (n, n, n), (1.0, 1.0, 1.0)
    z, y, x = grid_coords(shape, lengths)
    B = (np.zeros(shape), np.zeros(shape), -(z - 0.5))
    pts, count, status = ofl.trace(*B, np.array([[0.5, 0.5, 0.75], [0.5, 0.5, 0.5]]), 0.125, 10, 0.0, lengths)
    assert list(status) == [ofl.NULL, ofl.NULL]
    assert count[1] == 1 and np.all(np.isfinite(pts))
    assert abs(pts[count[0] - 1, 0, 2] - 0.5) < 0.126


def test_seed_outside_and_zero_steps():
    B, lengths = helix_case(5)
    pts, count, status = ofl.trace(*B, np.array([[1.2, 0.5, 0.5], [0.5, 0.5, 0.5]]), 0.1, 0, 0.0, lengths)
    assert list(count) == [1, 1] and list(status) == [ofl.EXIT, ofl.MAXSTEPS]
    assert np.array_equal(pts[0], [[1.2, 0.5, 0.5], [0.5, 0.5, 0.5]])


# --------------------------------------------------------------------- GPU
torch = pytest.importorskip("torch")


def smooth_field(shape, lengths, seed):
    """A smooth random field (a few sine modes per component) with nulls
    near some points."""
    z, y, x = grid_coords(shape, lengths)
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(3):
        F = np.zeros(shape)
        for _ in range(4):
            a, kx, ky, kz, ph = rng.normal(), *rng.integers(1, 4, 3), rng.uniform(0, 6.3)
            F += a * np.sin(kx * np.pi * x / lengths[0] + ph) * np.cos(ky * np.pi * y / lengths[1]) \
                * np.cos(kz * np.pi * z / lengths[2] + 0.5 * ph)
        out.append(F)
    return out


def gpu_trace(grid, B, seeds, ds, max_steps, bmin):
    from paper_1307_6720_amd.solver import Plan, trace_field_lines

    plan = Plan(grid, device="cuda:0")
    dev = [torch.from_numpy(np.ascontiguousarray(F)).to("cuda:0") for F in B]
    s = torch.from_numpy(np.ascontiguousarray(seeds, dtype=np.float64)).to("cuda:0")
    pts, cnt, st = trace_field_lines(plan, *dev, s, ds, max_steps, bmin)
    torch.cuda.synchronize()
    plan.close()
    return pts.cpu().numpy(), cnt.cpu().numpy(), st.cpu().numpy()


def compare_lines(got, want):
    pts, cnt, st = got
    wpts, wcnt, wst = want
    assert np.array_equal(cnt, wcnt) and np.array_equal(st, wst)
    worst = 0.0
    for l in range(len(cnt)):
        worst = max(worst, np.abs(pts[: cnt[l], l] - wpts[: cnt[l], l]).max())
    return worst


@pytest.mark.gpu
@pytest.mark.parametrize("shape,lengths,ds,bmin", [((33, 65, 129), (1.0, 1.3, 0.8), 0.011, 0.05),
                                                   ((17, 17, 17), (1.0, 1.0, 1.0), -0.03, 0.0),
                                                   ((65, 33, 17), (0.5, 2.0, 1.0), 0.02, 0.2)])
def test_gpu_field_lines_match_oracle(shape, lengths, ds, bmin):
    """Random smooth fields, 3000 seeds (a few outside the box): every line's
    point count and end status equal the oracle's exactly, and its points
    agree to rounding (the kernel evaluates the oracle's expressions in the
    same order)."""
    nz, ny, nx = shape
    B = smooth_field(shape, lengths, sum(shape))
    rng = np.random.default_rng(7)
    seeds = rng.uniform(-0.02, 1.02, size=(3000, 3)) * np.array(lengths)
    print(f"[lines] shape={shape} ds={ds} bmin={bmin}", flush=True)
    got = gpu_trace(synth.make_grid(nx, ny, nz, *lengths), B, seeds, ds, 150, bmin)
    want = ofl.trace(*B, seeds, ds, 150, bmin, lengths)
    assert (want[2] == ofl.EXIT).any() and (want[1] > 10).any()
    assert compare_lines(got, want) <= 1e-13


@pytest.mark.gpu
def test_gpu_field_lines_of_a_solved_equilibrium():
    """Lines of the 129^3 workload's recovered B from seeds on the base:
    equal to the oracle's lines on the same B; ds > 0 and ds < 0 from the
    same seeds are the lines of B and of -B."""
    from paper_1307_6720_amd import PREC_MIXED
    from paper_1307_6720_amd.solver import Plan, solve, trace_field_lines

    w = synth.workload("mhs-129")
    g = w.grid
    plan = Plan(g, device="cuda:0")
    print("[lines] solved 129^3", flush=True)
    res = solve(plan, torch.from_numpy(w.bz0).to("cuda:0"), w.model, precision=PREC_MIXED, rtol=1e-10)
    B = (res.Bx, res.By, res.Bz)
    rng = np.random.default_rng(11)
    seeds = np.concatenate([rng.uniform(0.05, 0.95, size=(400, 2)), np.full((400, 1), 0.0)], axis=1)
    sd = torch.from_numpy(seeds).to("cuda:0")
    fwd = [t.cpu().numpy() for t in trace_field_lines(plan, *B, sd, 0.004, 400, 1e-6)]
    neg = tuple(-t for t in B)
    back = [t.cpu().numpy() for t in trace_field_lines(plan, *neg, sd, 0.004, 400, 1e-6)]
    rev = [t.cpu().numpy() for t in trace_field_lines(plan, *B, sd, -0.004, 400, 1e-6)]
    Bh = [t.cpu().numpy() for t in B]
    plan.close()
    assert compare_lines(fwd, ofl.trace(*Bh, seeds, 0.004, 400, 1e-6, (g.lx, g.ly, g.lz))) <= 1e-13
    # -B with ds is B with -ds, operation for operation
    assert compare_lines(back, rev) == 0.0
    # lines from the base either return to it, leave through a side or the top,
    # or run to the cap; some of each kind the magnetogram's bipoles make
    assert (fwd[2] == ofl.EXIT).sum() > 0


@pytest.mark.gpu
def test_gpu_field_lines_edge_cases():
    from paper_1307_6720_amd import MHSError
    from paper_1307_6720_amd.solver import Plan, trace_field_lines

    shape, lengths = (9, 9, 9), (1.0, 1.0, 1.0)
    B = [torch.from_numpy(F).to("cuda:0") for F in helix_case(9)[0]]
    plan = Plan(synth.make_grid(9, 9, 9), device="cuda:0")
    print("[lines] edge cases", flush=True)
    empty = torch.zeros((0, 3), dtype=torch.float64, device="cuda:0")
    pts, cnt, st = trace_field_lines(plan, *B, empty, 0.1, 5)
    assert pts.shape == (6, 0, 3) and cnt.numel() == 0
    seeds = torch.tensor([[0.5, 0.5, 0.5], [-1.0, 0.5, 0.5]], dtype=torch.float64, device="cuda:0")
    pts, cnt, st = trace_field_lines(plan, *B, seeds, 0.1, 0)
    assert cnt.tolist() == [1, 1] and st.tolist() == [ofl.MAXSTEPS, ofl.EXIT]
    for bad in (dict(ds=0.0), dict(ds=float("nan")), dict(bmin=-1.0)):
        kw = dict(ds=0.1, bmin=0.0)
        kw.update(bad)
        with pytest.raises(MHSError):
            trace_field_lines(plan, *B, seeds, kw["ds"], 3, kw["bmin"])
    torch.cuda.synchronize()
    plan.close()
