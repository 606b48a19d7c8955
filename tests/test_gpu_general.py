"""The general elliptic problem of Section 2.2 on the GPU (mhs_solve_general,
mhs_solve_face) against the oracle: a fixed number of V-cycles equals the
oracle's multigrid (3D grids whose steps halve every axis, keep z, or keep x
and y; every face of a box), converged solutions equal the dense solve on
tiny grids and the exact solve of (8) when the general form reduces to it,
face problems feed the interior solve as Dirichlet data, and the error
paths of the C ABI.
"""

import numpy as np
import pytest

import synth
from oracle import dense, exact, ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1307_6720_amd import PLAN_GENERAL, PREC_FP64, PREC_MIXED, MHSError  # noqa: E402
from paper_1307_6720_amd import _lib  # noqa: E402
from paper_1307_6720_amd.solver import Plan, make_opts  # noqa: E402

DEV = torch.device("cuda:0")


def rel(a, b):
    d = np.abs(b).max()
    return float(np.abs(a - b).max() / (d if d > 0 else 1.0))


def coefficients(shape, lengths, seed):
    return synth.general_problem(shape, lengths, seed)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def plans():
    cache = {}

    def get(dims, lengths=(1.0, 1.0, 1.0)):
        key = (dims, lengths)
        if key not in cache:
            nx, ny, nz = dims
            cache[key] = Plan(synth.make_grid(nx, ny, nz, *lengths), PREC_FP64 | PLAN_GENERAL, device=DEV)
        return cache[key]

    yield get
    for p in cache.values():
        p.close()


@pytest.mark.parametrize("dims,lengths,cycles", [((33, 33, 33), (1.0, 1.0, 1.0), 1), ((33, 33, 33), (1.0, 1.0, 1.0), 3),
                                                 ((65, 33, 17), (1.0, 1.0, 1.0), 2),
                                                 ((9, 9, 65), (1.0, 1.0, 1.0), 2),
                                                 ((17, 33, 9), (0.5, 1.0, 0.5), 2)])
def test_general_fixed_cycles_match_the_oracle(plans, dims, lengths, cycles):
    """(65, 33, 17) keeps z on its first steps, (9, 9, 65) keeps x and y."""
    nx, ny, nz = dims
    print(f"[general] fixed cycles {dims} x{cycles}", flush=True)
    shape = (nz, ny, nx)
    a, b, c, u = coefficients(shape, lengths, 11)
    want, st, cyc, *_ = ref.gen_mg(u, a, b, c, rtol=-1.0, max_cycles=cycles, lengths=lengths)
    assert st == ref.OK and cyc == cycles
    plan = plans(dims, lengths)
    ud = dev(u)
    info = plan.solve_general(dev(a), dev(b), dev(c), ud, make_opts(rtol=1e-300, max_cycles=cycles),
                              raise_on_error=False)
    assert info.status == _lib.ERR_NO_CONVERGENCE and info.cycles == cycles
    got = ud.cpu().numpy()
    assert rel(got, want) < 1e-12, rel(got, want)
    inner = (slice(1, -1),) * 3
    mask = np.ones(shape, bool)
    mask[inner] = False
    assert np.array_equal(got[mask], u[mask])


FACES = [(_lib.FACE_BASE, "xy"), (_lib.FACE_TOP, "xy"), (_lib.FACE_XLO, "yz"), (_lib.FACE_XHI, "yz"),
         (_lib.FACE_YLO, "xz"), (_lib.FACE_YHI, "xz")]


def face_view(P, face):
    """The face of a (nz, ny, nx) array as a (n2, n1) view, first face
    coordinate fastest."""
    return {_lib.FACE_BASE: P[0], _lib.FACE_TOP: P[-1], _lib.FACE_XLO: P[:, :, 0], _lib.FACE_XHI: P[:, :, -1],
            _lib.FACE_YLO: P[:, 0, :], _lib.FACE_YHI: P[:, -1, :]}[face]


@pytest.mark.parametrize("face,axes", FACES)
def test_face_fixed_cycles_match_the_oracle(plans, face, axes):
    dims, lengths = (33, 17, 65), (1.0, 0.5, 2.0)
    nx, ny, nz = dims
    print(f"[general] face {face} ({axes})", flush=True)
    L = {"x": lengths[0], "y": lengths[1], "z": lengths[2]}
    flen = (L[axes[0]], L[axes[1]])
    plan = plans(dims, lengths)
    fshape = plan.face_shape(face)
    a, b, c, _ = coefficients(fshape, flen, 12)
    rng = np.random.default_rng(13)
    P = rng.normal(size=(nz, ny, nx))
    uf = face_view(P, face).copy()
    uf[1:-1, 1:-1] = 0.0
    want, st, cyc, *_ = ref.gen_mg(uf, a, b, c, rtol=-1.0, max_cycles=2, lengths=flen, planar=True)
    assert st == ref.OK
    Pd = dev(P)
    info = plan.solve_face(face, dev(a), dev(b), dev(c), Pd, make_opts(rtol=1e-300, max_cycles=2),
                           raise_on_error=False)
    assert info.status == _lib.ERR_NO_CONVERGENCE and info.cycles == 2
    got = Pd.cpu().numpy()
    assert rel(face_view(got, face), want) < 1e-12
    # nothing but the face's interior nodes changed
    keep = np.ones(P.shape, bool)
    fv = face_view(keep, face)
    fv[1:-1, 1:-1] = False
    assert np.array_equal(got[keep], P[keep])


@pytest.mark.parametrize("dims,lengths", [((5, 9, 9), (1.0, 0.5, 1.0)), ((17, 9, 5), (2.0, 1.0, 0.5))])
def test_general_converged_equals_dense(plans, dims, lengths):
    nx, ny, nz = dims
    shape = (nz, ny, nx)
    a, b, c, u = coefficients(shape, lengths, 14)
    plan = plans(dims, lengths)
    ud = dev(u)
    info = plan.solve_general(dev(a), dev(b), dev(c), ud, make_opts(rtol=1e-13, max_cycles=100))
    assert info.status == 0
    assert rel(ud.cpu().numpy(), dense.general(a, b, c, u, lengths)) < 1e-11


def test_general_reduces_to_equation_8(plans):
    """a = 1, b = alpha^2, c = 0 with the base plane of (11): the exact
    solution of (8) with xi = 0 (65^3, every node within 1e-10)."""
    w = synth.workload("mhs-129", dims=(65, 65, 65))
    g = w.grid
    alpha = 0.8
    want = exact.solve(w.bz0, g.nz, np.zeros(g.nz), alpha, g.lx, g.ly, g.lz)
    u = np.zeros(g.shape)
    u[0] = want[0]
    plan = plans((65, 65, 65))
    ud = dev(u)
    ones = torch.ones(g.shape, dtype=torch.float64, device=DEV)
    info = plan.solve_general(ones, ones * alpha**2, torch.zeros_like(ones), ud, make_opts(rtol=1e-12))
    assert info.status == 0 and info.cycles <= 15
    assert rel(ud.cpu().numpy(), want) < 1e-10


def test_faces_feed_the_interior_solve(plans):
    """Elliptic problems on every face but the base, then (11) on the base
    and (8) with the faces as given Dirichlet data: the result equals the
    oracle's face solves followed by its multigrid of (8) with the same
    faces."""
    dims = (33, 33, 33)
    nx, ny, nz = dims
    w = synth.workload("mhs-129", dims=dims)
    m = w.model
    plan = plans(dims)
    P = np.zeros((nz, ny, nx))
    Pd = dev(P)
    for face, axes in FACES[1:]:
        fshape = plan.face_shape(face)
        a, b, c, _ = coefficients(fshape, (1.0, 1.0), 20 + face)
        c = 0.05 * c
        uf = face_view(P, face).copy()
        want, st, *_ = ref.gen_mg(uf, a, b, c, rtol=1e-13, max_cycles=100, planar=True)
        assert st == ref.OK
        face_view(P, face)[...] = want
        plan.solve_face(face, dev(a), dev(b), dev(c), Pd, make_opts(rtol=1e-13))
    assert rel(Pd.cpu().numpy(), P) < 1e-11
    # base (11), then (8) with the given faces
    opts2 = make_opts(rtol=1e-13, faces_given=True)
    plan.solve_boundary(dev(w.bz0), Pd, opts2)
    plan.solve_interior(m, Pd, make_opts(rtol=1e-12, faces_given=True))
    P0, st, *_ = ref.mg2(w.bz0, rtol=1e-13, max_cycles=100, P0=P[0], keep_edges=True)
    assert st == ref.OK
    P[0] = P0
    Pw, st3, cyc, relres = ref.mg3(P, m.xi, m.alpha, rtol=1e-12, max_cycles=100)[:4]
    assert st3 == ref.OK
    assert rel(Pd.cpu().numpy(), Pw) < 1e-9


def test_general_error_paths(plans):
    dims = (17, 17, 17)
    shape = (17, 17, 17)
    plan = plans(dims)
    a, b, c, u = coefficients(shape, (1.0, 1.0, 1.0), 30)
    ad, bd, cd, ud = dev(a), dev(b), dev(c), dev(u)
    with pytest.raises(MHSError) as e:
        plan.solve_general(ad, bd, cd, ud, make_opts(PREC_MIXED))
    assert e.value.code == _lib.ERR_UNSUPPORTED
    a0 = a.copy()
    a0[8, 8, 8] = 0.0
    with pytest.raises(MHSError) as e:
        plan.solve_general(dev(a0), bd, cd, ud)
    assert e.value.code == _lib.ERR_INVALID_ARG
    # the 3^3 coarsest grid of the unit cube bounds b/a below 12
    with pytest.raises(MHSError) as e:
        plan.solve_general(ad, torch.full_like(bd, 12.5), cd, ud)
    assert e.value.code == _lib.ERR_INDEFINITE
    with pytest.raises(ValueError):
        plan.solve_face(7, ad[0], bd[0], cd[0], ud)
    plain = Plan(synth.make_grid(17, 17, 17), PREC_FP64, device=DEV)
    with pytest.raises(MHSError) as e:
        plain.solve_general(ad, bd, cd, ud)
    assert e.value.code == _lib.ERR_UNSUPPORTED
    plain.close()
