"""C-ABI checks that need no GPU: the library loads, exports every entry
point include/mhs.h declares, and validates grids and options on the host
before any device work."""

import ctypes as C
import os
import re

import pytest

from paper_1307_6720_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mhs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mhs_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_path():
    names = declared_functions()
    for required in ("mhs_solve_boundary", "mhs_solve_interior", "mhs_fields", "mhs_workspace_bytes",
                     "mhs_plan_create", "mhs_batch_step"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_defaults():
    L = _lib.lib()
    assert L.mhs_version() >= 10000
    o = _lib.Opts()
    L.mhs_default_opts(C.byref(o))
    assert (o.precision, o.max_cycles, o.nu1, o.nu2, o.inner_cycles) == (_lib.PREC_FP64, 100, 2, 2, 3)
    assert o.rtol == 1e-10


@pytest.mark.parametrize("args", [
    (None, 8, 8, 33, 33, 33, 1, 0, 32),   # NULL pointer
    (8, 8, 8, 2, 33, 33, 1, 0, 32),       # nx < 3
    (8, 8, 8, 33, 33, 33, 0, 0, 32),      # no request
    (8, 8, 8, 33, 33, 33, 1, 2, 32),      # no such tile
    (8, 8, 8, 33, 33, 33, 1, 0, 0),       # kz < 1
])
def test_pattern_probe_rejects_bad_arguments_on_the_host(args):
    """The access-pattern reference checks its arguments before any device
    work (the pointers below are never dereferenced)."""
    L = _lib.lib()
    ptrs = [None if v is None else C.c_void_p(v) for v in args[:3]]
    assert L.mhs_probe_smoother_pattern(*ptrs, *args[3:], None) == _lib.ERR_INVALID_ARG
    assert b"probe" in L.mhs_last_error() or b"NULL" in L.mhs_last_error()


def ws_bytes(nx, ny, nz, prec=3, lengths=(1.0, 1.0, 1.0)):
    g = _lib.Grid(nx, ny, nz, *lengths)
    n = C.c_size_t(0)
    code = _lib.lib().mhs_workspace_bytes(C.byref(g), prec, C.byref(n))
    return code, n.value


@pytest.mark.parametrize("dims", [(33, 33, 33), (257, 257, 257), (513, 513, 257), (129, 129, 65), (65, 17, 9)])
def test_workspace_sizes(dims):
    code, n = ws_bytes(*dims)
    assert code == _lib.MHS_OK
    N = dims[0] * dims[1] * dims[2]
    # at least the FP64 twin + FP32 correction, residual and twin on the finest grid
    assert n >= N * (8 + 3 * 4)
    # and not much more than two of those
    assert n < 2.2 * N * (8 + 3 * 4) + (8 << 20)
    c64, n64 = ws_bytes(*dims, prec=1)
    assert c64 == _lib.MHS_OK and n64 < n


@pytest.mark.parametrize("dims,code", [((32, 33, 33), _lib.ERR_GRID), ((33, 33, 3), _lib.ERR_GRID),
                                       ((33, 34, 33), _lib.ERR_GRID), ((4097, 5, 5), _lib.ERR_GRID),
                                       # over 2e9 nodes (32-bit node indices)
                                       ((32769, 16385, 5), _lib.ERR_GRID)])
def test_bad_grids_rejected(dims, code):
    got, _ = ws_bytes(*dims)
    assert got == code
    assert _lib.lib().mhs_last_error()


def test_bad_lengths_and_precisions_rejected():
    assert ws_bytes(33, 33, 33, lengths=(1.0, -1.0, 1.0))[0] == _lib.ERR_INVALID_ARG
    assert ws_bytes(33, 33, 33, prec=0)[0] == _lib.ERR_INVALID_ARG
    assert ws_bytes(33, 33, 33, prec=4)[0] == _lib.ERR_INVALID_ARG


def test_null_arguments_rejected():
    L = _lib.lib()
    assert L.mhs_workspace_bytes(None, 1, None) == _lib.ERR_INVALID_ARG
    assert L.mhs_solve_boundary(None, None, None, None, None, None) == _lib.ERR_INVALID_ARG
    assert L.mhs_solve_equilibrium(None, None, None, None, None, None, None, None, None, None, None, None, None,
                                   None) == _lib.ERR_INVALID_ARG
    assert L.mhs_plan_destroy(None) == _lib.MHS_OK
    assert L.mhs_trace_field_lines(None, None, None, None, None, 1, 0.1, 1, 0.0, None, None, None,
                                   None) == _lib.ERR_INVALID_ARG


def test_plan_create_rejects_small_or_misaligned_workspace():
    L = _lib.lib()
    g = _lib.Grid(33, 33, 33, 1.0, 1.0, 1.0)
    h = C.c_void_p()
    # workspace validation happens before any device call
    assert L.mhs_plan_create(C.byref(g), 3, C.c_void_p(256), 1024, C.byref(h)) == _lib.ERR_WORKSPACE
    _, n = ws_bytes(33, 33, 33)
    assert L.mhs_plan_create(C.byref(g), 3, C.c_void_p(4096 + 8), n, C.byref(h)) == _lib.ERR_WORKSPACE


def test_noalloc_solve_refuses_grids_past_its_array():
    """The interior solve without allocation holds its hierarchy in a fixed
    48 MiB device array: a grid whose workspace does not fit (257^3) is
    refused on the host before any device call, and so are bad arguments."""
    L = _lib.lib()
    o = _lib.Opts()
    L.mhs_default_opts(C.byref(o))
    xi = (C.c_double * 257)()
    m = _lib.Model(0.0, xi, None, None, None, 1.0, 1.0)
    fake = C.c_void_p(1 << 20)  # never dereferenced: the size check comes first
    for prec in (_lib.PREC_FP64, _lib.PREC_MIXED):
        o.precision = prec
        g = _lib.Grid(257, 257, 257, 1.0, 1.0, 1.0)
        assert L.mhs_solve_interior_noalloc(C.byref(g), C.byref(m), fake, C.byref(o), None,
                                            None) == _lib.ERR_WORKSPACE
        assert b"scratch" in L.mhs_last_error()
    g = _lib.Grid(129, 129, 129, 1.0, 1.0, 1.0)
    assert L.mhs_solve_interior_noalloc(C.byref(g), C.byref(m), None, C.byref(o), None, None) == _lib.ERR_INVALID_ARG
    bad = _lib.Grid(32, 33, 33, 1.0, 1.0, 1.0)
    assert L.mhs_solve_interior_noalloc(C.byref(bad), C.byref(m), fake, C.byref(o), None, None) == _lib.ERR_GRID
    # the largest grid it serves fits with either precision
    for prec in (_lib.PREC_FP64, _lib.PREC_MIXED):
        code, n = ws_bytes(129, 129, 129, prec=prec)
        assert code == _lib.MHS_OK and n - 256 <= 48 << 20


def test_request_bytes_counts_workspace_and_arrays():
    for dims in ((33, 33, 33), (257, 257, 257), (129, 129, 65)):
        g = _lib.Grid(*dims, 1.0, 1.0, 1.0)
        n = C.c_size_t(0)
        assert _lib.lib().mhs_request_bytes(C.byref(g), 3, C.byref(n)) == _lib.MHS_OK
        _, ws = ws_bytes(*dims)
        nx, ny, nz = dims
        assert n.value == ws + 8 * (6 * nx * ny * nz + nx * ny)
    bad = _lib.Grid(32, 33, 33, 1.0, 1.0, 1.0)
    assert _lib.lib().mhs_request_bytes(C.byref(bad), 3, C.byref(C.c_size_t())) == _lib.ERR_GRID
    assert _lib.lib().mhs_batch_bytes_in_use(None, None) == _lib.ERR_INVALID_ARG


torch = pytest.importorskip("torch")


def test_binding_rejects_wrong_arrays_before_the_c_call():
    """The C ABI takes bare pointers; the torch binding checks dtype, shape,
    contiguity and device of every array first (no GPU needed: the check
    raises before any library call)."""
    from paper_1307_6720_amd import solver

    good = torch.zeros((3, 4, 5), dtype=torch.float64)
    solver.check_array(good, (3, 4, 5), torch.float64, "cpu", "P")
    for t, why in ((good.float(), "float64"), (good[:, :, :4], "shape"), (good.transpose(0, 2).contiguous(), "shape"),
                   (torch.zeros((5, 4, 3), dtype=torch.float64).transpose(0, 2), "contiguous"),
                   (good.numpy(), "tensor")):
        with pytest.raises(ValueError, match=why):
            solver.check_array(t, (3, 4, 5), torch.float64, "cpu", "P")
    with pytest.raises(ValueError, match="must be on"):
        solver.check_array(good, (3, 4, 5), torch.float64, "cuda:0", "P")
    # a Plan's entry points run the checks before the C call
    plan = solver.Plan.__new__(solver.Plan)
    plan.cgrid = _lib.Grid(5, 4, 3, 1.0, 1.0, 1.0)
    plan.device = torch.device("cpu")
    plan.h = None
    bz = torch.zeros((4, 5), dtype=torch.float64)
    with pytest.raises(ValueError, match="bz0"):
        plan.solve_boundary(bz.float(), good)
    with pytest.raises(ValueError, match="P"):
        plan.solve_boundary(bz, good[:2])
    with pytest.raises(ValueError, match="P"):
        plan.solve_interior(None, good.float())
    with pytest.raises(ValueError, match="Bx"):
        plan.fields(None, good, out=(good[:1],) + tuple(torch.zeros_like(good) for _ in range(4)))
    with pytest.raises(ValueError, match="five"):
        plan.fields(None, good, out=(good,) * 4)
