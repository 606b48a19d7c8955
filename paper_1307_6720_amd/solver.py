"""Torch-level interface to libmhs: plans, solves and field recovery.

PyTorch provides device memory and streams only; every step of the solve runs
in the HIP library through the C ABI declared in include/mhs.h.
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import PREC_FP64, PREC_MIXED, MHSError, check


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _same_device(a, b):
    a, b = torch.device(a), torch.device(b)
    if a.type != b.type:
        return False
    if a.type != "cuda":
        return True
    ia = torch.cuda.current_device() if a.index is None else a.index
    ib = torch.cuda.current_device() if b.index is None else b.index
    return ia == ib


def check_array(t, shape, dtype, device, name):
    """Raise ValueError unless `t` is a contiguous tensor of `dtype` and
    `shape` on `device`.  The C ABI takes bare pointers and cannot check
    sizes, so every array is checked here before its pointer is passed."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if not _same_device(t.device, device):
        raise ValueError(f"{name} must be on {device}, got {t.device}")


def make_opts(precision=PREC_FP64, rtol=1e-10, max_cycles=100, nu1=2, nu2=2, inner_cycles=None,
              warm_start=False, check_every=0, faces_given=False, graph=False):
    o = _lib.Opts()
    _lib.lib().mhs_default_opts(C.byref(o))
    o.precision = precision
    o.rtol = rtol
    o.max_cycles = max_cycles
    o.nu1 = nu1
    o.nu2 = nu2
    if inner_cycles is not None:  # None keeps the library's default
        o.inner_cycles = inner_cycles
    o.warm_start = 1 if warm_start else 0
    o.check_every = check_every
    o.faces = _lib.FACES_GIVEN if faces_given else _lib.FACES_ZERO
    o.graph = 1 if graph else 0
    return o


class _ModelArgs:
    """Keeps the host arrays of a model alive while the C struct points at them."""

    def __init__(self, alpha, xi, dxi=None, pb=None, rhob=None, mu0=1.0, g=1.0):
        self.arrays = []

        def arr(a):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=np.float64)
            self.arrays.append(a)
            return a.ctypes.data_as(C.POINTER(C.c_double))

        self.c = _lib.Model(float(alpha), arr(xi), arr(dxi), arr(pb), arr(rhob), float(mu0), float(g))

    @classmethod
    def of(cls, model):
        if model is None:
            return None
        return cls(model.alpha, model.xi, model.dxi, model.pb, model.rhob, model.mu0, model.g)


@dataclass
class GridSpec:
    nx: int
    ny: int
    nz: int
    lx: float = 1.0
    ly: float = 1.0
    lz: float = 1.0

    def c(self):
        return _lib.Grid(self.nx, self.ny, self.nz, self.lx, self.ly, self.lz)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)


def workspace_bytes(grid, precisions=PREC_FP64 | PREC_MIXED):
    g = _grid(grid)
    n = C.c_size_t(0)
    check(_lib.lib().mhs_workspace_bytes(C.byref(g), precisions, C.byref(n)))
    return n.value


def request_bytes(grid, precisions=PREC_FP64 | PREC_MIXED):
    """Device bytes one served request holds: workspace, bz0, P and the
    five field outputs (mhs_request_bytes)."""
    g = _grid(grid)
    n = C.c_size_t(0)
    check(_lib.lib().mhs_request_bytes(C.byref(g), precisions, C.byref(n)))
    return n.value


def check_model(grid, model):
    """Host-only validation of a model on a grid (no device needed).
    Returns (lambda_0, levels): the smallest eigenvalue of
    -[(1-xi)(d2x+d2y)+d2z] on the grid, and the number of 3D multigrid levels
    the solve uses.  Raises MHSError (NOT_ELLIPTIC, INDEFINITE, ...)."""
    g = _grid(grid)
    m = _ModelArgs.of(model)
    lam = C.c_double()
    lv = C.c_int32()
    check(_lib.lib().mhs_check_model(C.byref(g), C.byref(m.c), C.byref(lam), C.byref(lv)))
    return lam.value, lv.value


def solve_interior_noalloc(grid, model, P, opts=None, raise_on_error=True):
    """Equation (8) in place on P's device without a plan or workspace
    (mhs_solve_interior_noalloc): the library's fixed scratch array holds
    the hierarchy, so grids up to 129^3 only; same results as
    Plan.solve_interior.  Plane 0 of P must already hold the base solution."""
    g = _grid(grid)
    if not isinstance(P, torch.Tensor) or P.device.type != "cuda":
        raise ValueError("P must be a CUDA tensor")
    check_array(P, (g.nz, g.ny, g.nx), torch.float64, P.device, "P")
    opts = opts or make_opts()
    m = _ModelArgs.of(model)
    info = _lib.Info()
    with torch.cuda.device(P.device):
        code = _lib.lib().mhs_solve_interior_noalloc(C.byref(g), C.byref(m.c), _ptr(P), C.byref(opts),
                                                     C.byref(info), _stream(P.device))
    if raise_on_error:
        check(code)
    return info


def _grid(grid):
    if isinstance(grid, _lib.Grid):
        return grid
    return _lib.Grid(int(grid.nx), int(grid.ny), int(grid.nz), float(grid.lx), float(grid.ly), float(grid.lz))


class Plan:
    """A multigrid plan over a torch-allocated workspace on one device."""

    def __init__(self, grid, precisions=PREC_FP64 | PREC_MIXED, device="cuda:0", workspace=None):
        self.grid = grid
        self.cgrid = _grid(grid)
        self.device = torch.device(device)
        self.precisions = precisions
        self.ws_bytes = workspace_bytes(grid, precisions)
        with torch.cuda.device(self.device):
            if workspace is None:
                workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
            if workspace.numel() < self.ws_bytes:
                raise ValueError("workspace too small")
            self.ws = workspace
            h = C.c_void_p()
            check(_lib.lib().mhs_plan_create(C.byref(self.cgrid), precisions, C.c_void_p(workspace.data_ptr()),
                                             workspace.numel(), C.byref(h)))
        self.h = h

    @property
    def shape(self):
        return (self.cgrid.nz, self.cgrid.ny, self.cgrid.nx)

    def close(self):
        if getattr(self, "h", None):
            _lib.lib().mhs_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def levels(self, space=3):
        n = C.c_int32()
        check(_lib.lib().mhs_plan_levels(self.h, space, C.byref(n)))
        return n.value

    def bottom_level(self, space=3):
        n = C.c_int32()
        check(_lib.lib().mhs_plan_bottom_level(self.h, space, C.byref(n)))
        return n.value

    def level_shape(self, space, level):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        check(_lib.lib().mhs_plan_level_dims(self.h, space, level, C.byref(a), C.byref(b), C.byref(c)))
        return (c.value, b.value, a.value) if space == 3 else (b.value, a.value)

    def _check(self, t, shape, name, dtype=torch.float64):
        check_array(t, shape, dtype, self.device, name)

    def _check_fields(self, ts, names):
        for t, n in zip(ts, names):
            self._check(t, self.shape, n)

    # ---- the three steps of the procedure ------------------------------------
    def solve_boundary(self, bz0, P, opts=None, raise_on_error=True):
        """Multigrid solve of equation (11); writes plane 0 of P."""
        self._check(bz0, self.shape[1:], "bz0")
        self._check(P, self.shape, "P")
        opts = opts or make_opts()
        info = _lib.Info()
        with torch.cuda.device(self.device):
            code = _lib.lib().mhs_solve_boundary(self.h, _ptr(bz0), _ptr(P), C.byref(opts), C.byref(info),
                                                 _stream(self.device))
        if raise_on_error:
            check(code)
        return info

    def solve_interior(self, model, P, opts=None, raise_on_error=True):
        """Multigrid solve of equation (8) in place (FP64 or mixed)."""
        self._check(P, self.shape, "P")
        opts = opts or make_opts()
        m = _ModelArgs.of(model)
        info = _lib.Info()
        with torch.cuda.device(self.device):
            code = _lib.lib().mhs_solve_interior(self.h, C.byref(m.c), _ptr(P), C.byref(opts), C.byref(info),
                                                 _stream(self.device))
        if raise_on_error:
            check(code)
        return info

    def solve_equilibrium(self, bz0, model, P, out=None, opts2d=None, opts3d=None, raise_on_error=True):
        """Equations (11) and (8) and the field recovery in one library call
        (mhs_solve_equilibrium): the results of solve_boundary,
        solve_interior and fields in turn, with fewer host round trips.
        out: five tensors (Bx, By, Bz, p, rho), or None for no recovery.
        Returns (info2d, info3d)."""
        self._check(bz0, self.shape[1:], "bz0")
        self._check(P, self.shape, "P")
        if out is not None:
            out = tuple(out)
            if len(out) != 5:
                raise ValueError("out must hold five tensors (Bx, By, Bz, p, rho)")
            self._check_fields(out, ("Bx", "By", "Bz", "p", "rho"))
        o2 = opts2d or make_opts()
        o3 = opts3d or make_opts()
        m = _ModelArgs.of(model)
        i2, i3 = _lib.Info(), _lib.Info()
        fp = [_ptr(t) for t in out] if out is not None else [None] * 5
        with torch.cuda.device(self.device):
            code = _lib.lib().mhs_solve_equilibrium(self.h, C.byref(m.c), _ptr(bz0), _ptr(P), *fp, C.byref(o2),
                                                    C.byref(o3), C.byref(i2), C.byref(i3), _stream(self.device))
        if raise_on_error:
            check(code)
        return i2, i3

    # ---- the general elliptic problem of Section 2.2 ---------------------------
    def solve_general(self, a, b, c, u, opts=None, raise_on_error=True):
        """a lap u + b u = c on the plan's 3D grid (per-node FP64 a, b, c of
        the grid's shape); u's boundary values are the Dirichlet data, its
        interior receives the solution.  The plan needs PLAN_GENERAL."""
        for t, n in ((a, "a"), (b, "b"), (c, "c"), (u, "u")):
            self._check(t, self.shape, n)
        opts = opts or make_opts()
        info = _lib.Info()
        with torch.cuda.device(self.device):
            code = _lib.lib().mhs_solve_general(self.h, _ptr(a), _ptr(b), _ptr(c), _ptr(u), C.byref(opts),
                                                C.byref(info), _stream(self.device))
        if raise_on_error:
            check(code)
        return info

    def face_shape(self, face):
        """Shape (n2, n1) of the coefficient arrays of a face problem."""
        nz, ny, nx = self.shape
        if face in (_lib.FACE_BASE, _lib.FACE_TOP):
            return (ny, nx)
        if face in (_lib.FACE_XLO, _lib.FACE_XHI):
            return (nz, ny)
        if face in (_lib.FACE_YLO, _lib.FACE_YHI):
            return (nz, nx)
        raise ValueError("face must be one of FACE_BASE .. FACE_YHI")

    def solve_face(self, face, a, b, c, P, opts=None, raise_on_error=True):
        """a lap u + b u = c on one face of the box (2D Laplacian in the
        face's coordinates), the face's edges in P as Dirichlet data; the
        interior nodes of that face of P receive the solution."""
        fs = self.face_shape(face)
        for t, n in ((a, "a"), (b, "b"), (c, "c")):
            self._check(t, fs, n)
        self._check(P, self.shape, "P")
        opts = opts or make_opts()
        info = _lib.Info()
        with torch.cuda.device(self.device):
            code = _lib.lib().mhs_solve_face(self.h, int(face), _ptr(a), _ptr(b), _ptr(c), _ptr(P), C.byref(opts),
                                             C.byref(info), _stream(self.device))
        if raise_on_error:
            check(code)
        return info

    def fields(self, model, P, out=None):
        """B, p, rho by central differences; returns (Bx, By, Bz, p, rho)."""
        self._check(P, self.shape, "P")
        if out is None:
            out = tuple(torch.empty_like(P) for _ in range(5))
        out = tuple(out)
        if len(out) != 5:
            raise ValueError("out must hold five tensors (Bx, By, Bz, p, rho)")
        self._check_fields(out, ("Bx", "By", "Bz", "p", "rho"))
        m = _ModelArgs.of(model)
        with torch.cuda.device(self.device):
            check(_lib.lib().mhs_fields(self.h, C.byref(m.c), _ptr(P), *[_ptr(t) for t in out],
                                        _stream(self.device)))
        return out

    def diagnostics(self, model, Bx, By, Bz, p, rho, out=None):
        """Residuals of equations (1)-(3) for the given fields: returns
        (jx, jy, jz, fres, divb) with j = curl B / mu0, fres the magnitude of
        the force-balance residual and divb = div B (zero on the side and top
        faces)."""
        self._check_fields((Bx, By, Bz, p, rho), ("Bx", "By", "Bz", "p", "rho"))
        if out is None:
            out = tuple(torch.empty_like(Bx) for _ in range(5))
        out = tuple(out)
        if len(out) != 5:
            raise ValueError("out must hold five tensors (jx, jy, jz, fres, divb)")
        self._check_fields(out, ("jx", "jy", "jz", "fres", "divb"))
        m = _ModelArgs.of(model)
        with torch.cuda.device(self.device):
            check(_lib.lib().mhs_diagnostics(self.h, C.byref(m.c), *[_ptr(t) for t in (Bx, By, Bz, p, rho)],
                                             *[_ptr(t) for t in out], _stream(self.device)))
        return out

    def trace_field_lines(self, Bx, By, Bz, seeds, ds, max_steps, bmin=0.0, out=None):
        """Field lines through `seeds` (torch float64 (nlines, 3) on the
        plan's device): returns (points, count, status) with points of shape
        (max_steps + 1, nlines, 3) (line l is points[:count[l], l]; later
        entries are not written), count and status int32 (nlines,); status
        0 = step cap, 1 = left the box, 2 = |B| <= bmin.  ds < 0 traces
        against B."""
        self._check_fields((Bx, By, Bz), ("Bx", "By", "Bz"))
        if not isinstance(seeds, torch.Tensor) or seeds.dim() != 2:
            raise ValueError("seeds must be a tensor of shape (nlines, 3)")
        n = seeds.shape[0]
        self._check(seeds, (n, 3), "seeds")
        if out is None:
            out = (torch.empty((max_steps + 1, n, 3), dtype=torch.float64, device=seeds.device),
                   torch.empty(n, dtype=torch.int32, device=seeds.device),
                   torch.empty(n, dtype=torch.int32, device=seeds.device))
        pts, cnt, st = out
        self._check(pts, (max_steps + 1, n, 3), "points")
        self._check(cnt, (n,), "count", torch.int32)
        self._check(st, (n,), "status", torch.int32)
        with torch.cuda.device(self.device):
            check(_lib.lib().mhs_trace_field_lines(self.h, _ptr(Bx), _ptr(By), _ptr(Bz), _ptr(seeds), n,
                                                   float(ds), int(max_steps), float(bmin), _ptr(pts), _ptr(cnt),
                                                   _ptr(st), _stream(self.device)))
        return pts, cnt, st

    # ---- measurement -----------------------------------------------------------
    def profile(self, enable=True, classes=None):
        """Time launches of the given classes (names from PROF_NAMES; all by
        default) with HIP events; enable=False turns profiling off."""
        mask = 0
        if enable:
            names = _lib.PROF_NAMES if classes is None else classes
            for n in names:
                mask |= 1 << _lib.PROF_NAMES.index(n)
        check(_lib.lib().mhs_profile_enable(self.h, mask))

    def profile_read(self, reset=False):
        """{class: (total_ms, launches, compulsory_bytes)} since the last reset."""
        out = {}
        for k, name in enumerate(_lib.PROF_NAMES):
            ms, n, b = C.c_double(), C.c_int64(), C.c_double()
            check(_lib.lib().mhs_profile_read(self.h, k, C.byref(ms), C.byref(n), C.byref(b), 0))
            out[name] = (ms.value, n.value, b.value)
        if reset:
            check(_lib.lib().mhs_profile_read(self.h, 0, None, None, None, 1))
        return out

    # ---- stage entry points (kernel-level checks) ----------------------------
    def _check_stage(self, space, level, precision, arrays):
        """arrays: (tensor or None, level offset, name); level offset 1 = the
        next coarser level's shape."""
        if space not in (2, 3) or precision not in (PREC_FP64, PREC_MIXED):
            raise ValueError("space must be 2 or 3 and precision MHS_PREC_FP64 or MHS_PREC_MIXED")
        dtype = torch.float64 if precision == PREC_FP64 else torch.float32
        for t, off, name in arrays:
            if t is not None:
                self._check(t, self.level_shape(space, level + off), name, dtype)

    def stage_smooth(self, model, space, level, u, f=None, nsweeps=1, precision=PREC_FP64, zero_guess=False):
        """nsweeps red-black sweeps on level `level`; zero_guess: the first
        sweep starts from u = 0, as the first sweep of a coarse-grid
        correction does (u's interior is not read; its boundary must be 0)."""
        self._check_stage(space, level, precision, ((u, 0, "u"), (f, 0, "f")))
        m = _ModelArgs.of(model)
        with torch.cuda.device(self.device):
            check(_lib.lib().mhs_stage_smooth(self.h, C.byref(m.c) if m else None, space, level, precision,
                                              _ptr(u), _ptr(f), nsweeps, 1 if zero_guess else 0,
                                              _stream(self.device)))
        return u

    def stage_restrict(self, model, space, level, u, f, fc, precision=PREC_FP64):
        self._check_stage(space, level, precision, ((u, 0, "u"), (f, 0, "f"), (fc, 1, "fc")))
        m = _ModelArgs.of(model)
        with torch.cuda.device(self.device):
            check(_lib.lib().mhs_stage_restrict(self.h, C.byref(m.c) if m else None, space, level, precision,
                                                _ptr(u), _ptr(f), _ptr(fc), _stream(self.device)))
        return fc

    def stage_correct_smooth(self, model, space, level, u, f, ec, precision=PREC_FP64, nsweeps=1):
        """u + I(ec) followed by nsweeps sweeps (the first fused with the
        interpolation)."""
        self._check_stage(space, level, precision, ((u, 0, "u"), (f, 0, "f"), (ec, 1, "ec")))
        m = _ModelArgs.of(model)
        with torch.cuda.device(self.device):
            check(_lib.lib().mhs_stage_correct_smooth(self.h, C.byref(m.c) if m else None, space, level,
                                                      precision, _ptr(u), _ptr(f), _ptr(ec), int(nsweeps),
                                                      _stream(self.device)))
        return u

    def stage_bottom(self, model, space, u, f, nu1=2, nu2=2, precision=PREC_FP64):
        # the bottom level depends on the model (uploaded by the call), so
        # the shape is checked against every level the plan has
        if space not in (2, 3) or precision not in (PREC_FP64, PREC_MIXED):
            raise ValueError("space must be 2 or 3 and precision MHS_PREC_FP64 or MHS_PREC_MIXED")
        shapes = [self.level_shape(space, l) for l in range(1, self.levels(space))]
        if not isinstance(u, torch.Tensor) or tuple(u.shape) not in shapes:
            raise ValueError(f"u must have the shape of a coarse level, one of {shapes}")
        dtype = torch.float64 if precision == PREC_FP64 else torch.float32
        self._check(u, tuple(u.shape), "u", dtype)
        self._check(f, tuple(u.shape), "f", dtype)
        m = _ModelArgs.of(model)
        lvl = C.c_int32()
        with torch.cuda.device(self.device):
            check(_lib.lib().mhs_stage_bottom(self.h, C.byref(m.c) if m else None, space, precision, _ptr(u),
                                              _ptr(f), nu1, nu2, C.byref(lvl), _stream(self.device)))
        return lvl.value

    def stage_residual_norm(self, model, space, level, u, f=None, precision=PREC_FP64):
        self._check_stage(space, level, precision, ((u, 0, "u"), (f, 0, "f")))
        m = _ModelArgs.of(model)
        out = C.c_double()
        with torch.cuda.device(self.device):
            check(_lib.lib().mhs_stage_residual_norm(self.h, C.byref(m.c) if m else None, space, level,
                                                     precision, _ptr(u), _ptr(f), C.byref(out),
                                                     _stream(self.device)))
        return out.value


@dataclass
class SolveResult:
    P: torch.Tensor
    Bx: torch.Tensor
    By: torch.Tensor
    Bz: torch.Tensor
    p: torch.Tensor
    rho: torch.Tensor
    info2d: dict
    info3d: dict


def solve(plan: Plan, bz0, model, precision=PREC_FP64, rtol=1e-10, rtol2d=None, max_cycles=100,
          inner_cycles=None, fields=True, out=None):
    """The whole path: (11) on the base, (8) in the interior, then B, p, rho.

    bz0: torch float64 (ny, nx) on the plan's device; model: synth.Model-like.
    """
    dev = plan.device
    shape = plan.shape
    if out is None:
        P = torch.empty(shape, dtype=torch.float64, device=dev)
        F = tuple(torch.empty(shape, dtype=torch.float64, device=dev) for _ in range(5)) if fields else None
    else:
        P, F = out[0], tuple(out[1:]) if fields else None
    o2 = make_opts(PREC_FP64, rtol if rtol2d is None else rtol2d, max_cycles)
    o3 = make_opts(precision, rtol, max_cycles, inner_cycles=inner_cycles)
    i2, i3 = plan.solve_equilibrium(bz0, model, P, F if fields else None, o2, o3)
    if not fields:
        F = (None,) * 5
    return SolveResult(P, *F, i2.as_dict(), i3.as_dict())


def diagnostics(plan: Plan, model, Bx, By, Bz, p, rho, out=None):
    """Residuals of equations (1)-(3) on the plan's grid (see Plan.diagnostics)."""
    return plan.diagnostics(model, Bx, By, Bz, p, rho, out)


def trace_field_lines(plan: Plan, Bx, By, Bz, seeds, ds, max_steps, bmin=0.0, out=None):
    """Field lines on the plan's grid (see Plan.trace_field_lines)."""
    return plan.trace_field_lines(Bx, By, Bz, seeds, ds, max_steps, bmin, out)
