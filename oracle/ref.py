"""ctypes binding of the oracle's C multigrid (mg_ref.c).

ORACLE -- test infrastructure, not the product.  Arrays are numpy float64,
C-contiguous, x fastest: 3D arrays have shape (nz, ny, nx), 2D (ny, nx).
Every function follows the passage cited in mg_ref.c; this file only
marshals arguments.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

OK, NO_CONVERGENCE, DIVERGED = 0, 1, 2
BAD_GRID, SINGULAR, NOMEM, INDEFINITE = -1, -2, -3, -4

_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    lib = C.CDLL(LIB)
    vp = C.c_void_p
    sig = {
        "ref_set_threads": (C.c_int, [C.c_int]),
        "ref_gen_mg": (C.c_int, [_ip, _dp, C.c_int, _dp, _dp, _dp, _dp, C.c_double, C.c_int, C.c_int, C.c_int,
                                 C.POINTER(C.c_int), C.POINTER(C.c_double), vp]),
        "ref_gen_levels": (C.c_int, [_ip, _dp, C.c_int]),
        "ref_gen_residual": (None, [_ip, _dp, C.c_int, _dp, _dp, _dp, _dp]),
        "ref_gen_normalise": (C.c_int, [_ip, C.c_int, _dp, _dp, _dp, _dp, _dp]),
        "ref_gen_rbgs": (None, [_ip, _dp, C.c_int, _dp, _dp, _dp, C.c_int]),
        "ref_gen_direct": (C.c_int, [_ip, _dp, C.c_int, _dp, _dp, _dp]),
        "ref_gen_inject": (None, [_ip, C.c_int, C.c_int, _dp, _dp]),
        "ref_levels3": (C.c_int, [_ip, _dp, _ip]),
        "ref_nlevels2": (C.c_int, [C.c_int, C.c_int]),
        "ref_residual3": (None, [_ip, _dp, _dp, C.c_double, _dp, vp, _dp]),
        "ref_norm3_interior": (C.c_double, [_ip, _dp]),
        "ref_rbgs3": (None, [_ip, _dp, _dp, C.c_double, _dp, vp, C.c_int]),
        "ref_restrict3": (None, [_ip, _dp, _dp]),
        "ref_prolong3": (None, [_ip, _dp, _dp]),
        "ref_restrict3_xy": (None, [_ip, _dp, _dp]),
        "ref_prolong3_xy": (None, [_ip, _dp, _dp]),
        "ref_restrict3_z": (None, [_ip, _dp, _dp]),
        "ref_prolong3_z": (None, [_ip, _dp, _dp]),
        "ref_direct3": (C.c_int, [_ip, _dp, _dp, C.c_double, _dp, vp]),
        "ref_mg3": (C.c_int, [_ip, _dp, _dp, C.c_double, _dp, C.c_double, C.c_int, C.c_int,
                              C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double), vp]),
        "ref_vcycle3_once": (C.c_int, [_ip, _dp, _dp, C.c_double, _dp, vp, C.c_int, C.c_int]),
        "ref_residual2": (None, [_ip, _dp, _dp, vp, _dp]),
        "ref_norm2_interior": (C.c_double, [_ip, _dp]),
        "ref_rbgs2": (None, [_ip, _dp, _dp, vp, C.c_int]),
        "ref_restrict2": (None, [_ip, _dp, _dp]),
        "ref_prolong2": (None, [_ip, _dp, _dp]),
        "ref_direct2": (C.c_int, [_ip, _dp, _dp, vp]),
        "ref_mg2": (C.c_int, [_ip, _dp, _dp, _dp, C.c_double, C.c_int, C.c_int, C.c_int,
                              C.POINTER(C.c_int), C.POINTER(C.c_double), vp]),
        "ref_mg2_edges": (C.c_int, [_ip, _dp, _dp, _dp, C.c_double, C.c_int, C.c_int, C.c_int,
                                    C.POINTER(C.c_int), C.POINTER(C.c_double), vp, C.c_int]),
        "ref_jacobi2": (None, [_ip, _dp, _dp, _dp, _dp]),
        "ref_solve": (C.c_int, [_ip, _dp, _dp, _dp, C.c_double, _dp, C.c_double, C.c_double,
                                C.c_int, C.c_int, C.c_int, _dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    # one thread unless asked (set_threads): test workers run side by side
    lib.ref_set_threads(1)
    _lib = lib
    return lib


def _n3(shape):
    nz, ny, nx = shape
    return np.array([nx, ny, nz], dtype=np.int32)


def _n2(shape):
    ny, nx = shape
    return np.array([nx, ny], dtype=np.int32)


def _h(shape, lengths):
    return np.array([l / (n - 1) for n, l in zip(shape[::-1], lengths)], dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


STEP_ALL, STEP_XY, STEP_Z = 0, 1, 2


def levels3(nx, ny, nz, lengths=(1.0, 1.0, 1.0)):
    """(number of 3D levels, [kind of each step l -> l+1]): STEP_ALL halves
    every axis, STEP_XY keeps z, STEP_Z keeps x and y."""
    keep = np.zeros(32, dtype=np.int32)
    L = _load().ref_levels3(np.array([nx, ny, nz], dtype=np.int32), _f64(lengths), keep)
    return L, [int(v) for v in keep[: max(L - 1, 0)]]


def nlevels3(nx, ny, nz, lengths=(1.0, 1.0, 1.0)):
    return levels3(nx, ny, nz, lengths)[0]


def nlevels2(nx, ny):
    return _load().ref_nlevels2(nx, ny)


# ---------------------------------------------------------------- 3D stages
def residual3(u, f, xi, alpha, lengths=(1.0, 1.0, 1.0)):
    """r = f - A u at interior nodes of (8); zero on boundary nodes."""
    u = _f64(u)
    f = None if f is None else _f64(f)
    r = np.zeros_like(u)
    _load().ref_residual3(_n3(u.shape), _h(u.shape, lengths), _f64(xi), alpha, u, _ptr(f), r)
    return r


def norm3_interior(r):
    r = _f64(r)
    return _load().ref_norm3_interior(_n3(r.shape), r)


def rbgs3(u, f, xi, alpha, nsweeps=1, lengths=(1.0, 1.0, 1.0)):
    """Return u after nsweeps red-black Gauss-Seidel sweeps (red first)."""
    u = _f64(u).copy()
    f = None if f is None else _f64(f)
    _load().ref_rbgs3(_n3(u.shape), _h(u.shape, lengths), _f64(xi), alpha, u, _ptr(f), nsweeps)
    return u


def restrict3(rf):
    rf = _f64(rf)
    nz, ny, nx = rf.shape
    fc = np.zeros(((nz - 1) // 2 + 1, (ny - 1) // 2 + 1, (nx - 1) // 2 + 1))
    _load().ref_restrict3(_n3(rf.shape), rf, fc)
    return fc


def prolong3(ec, uf):
    """Return uf + I(ec) on interior fine nodes (trilinear)."""
    ec = _f64(ec)
    uf = _f64(uf).copy()
    _load().ref_prolong3(_n3(ec.shape), ec, uf)
    return uf


def restrict3_xy(rf):
    """Full weighting within each plane (z kept)."""
    rf = _f64(rf)
    nz, ny, nx = rf.shape
    fc = np.zeros((nz, (ny - 1) // 2 + 1, (nx - 1) // 2 + 1))
    _load().ref_restrict3_xy(_n3(rf.shape), rf, fc)
    return fc


def prolong3_xy(ec, uf):
    """Return uf + I(ec) on interior fine nodes (bilinear within planes)."""
    ec = _f64(ec)
    uf = _f64(uf).copy()
    _load().ref_prolong3_xy(_n3(ec.shape), ec, uf)
    return uf


def restrict3_z(rf):
    """Full weighting along z only (x and y kept)."""
    rf = _f64(rf)
    nz, ny, nx = rf.shape
    fc = np.zeros(((nz - 1) // 2 + 1, ny, nx))
    _load().ref_restrict3_z(_n3(rf.shape), rf, fc)
    return fc


def prolong3_z(ec, uf):
    """Return uf + I(ec) on interior fine nodes (linear along z)."""
    ec = _f64(ec)
    uf = _f64(uf).copy()
    _load().ref_prolong3_z(_n3(ec.shape), ec, uf)
    return uf


def direct3(u, f, xi, alpha, lengths=(1.0, 1.0, 1.0)):
    """Exact dense solve of the interior unknowns; boundary values from u."""
    u = _f64(u).copy()
    f = None if f is None else _f64(f)
    st = _load().ref_direct3(_n3(u.shape), _h(u.shape, lengths), _f64(xi), alpha, u, _ptr(f))
    if st != OK:
        raise RuntimeError(f"ref_direct3 failed: {st}")
    return u


def vcycle3_once(u, f, xi, alpha, nu1=2, nu2=2, lengths=(1.0, 1.0, 1.0)):
    u = _f64(u).copy()
    f = None if f is None else _f64(f)
    st = _load().ref_vcycle3_once(_n3(u.shape), _f64(lengths), _f64(xi), alpha, u, _ptr(f), nu1, nu2)
    if st != OK:
        raise RuntimeError(f"ref_vcycle3_once failed: {st}")
    return u


def mg3(P, xi, alpha, rtol=1e-10, max_cycles=50, nu1=2, nu2=2, lengths=(1.0, 1.0, 1.0),
        history=False):
    """Multigrid solve of (8); P's boundary values are the Dirichlet data.

    Returns (P, status, cycles, relres[, hist])."""
    P = _f64(P).copy()
    cyc = C.c_int(0)
    rel = C.c_double(0.0)
    hist = np.zeros(max_cycles + 1)
    st = _load().ref_mg3(_n3(P.shape), _f64(lengths), _f64(xi), alpha, P, rtol, max_cycles,
                         nu1, nu2, C.byref(cyc), C.byref(rel), _ptr(hist))
    out = (P, st, cyc.value, rel.value)
    return out + (hist[: cyc.value + 1],) if history else out


# ---------------------------------------------------------------- 2D stages
def residual2(u, f, lengths=(1.0, 1.0)):
    u = _f64(u)
    f = None if f is None else _f64(f)
    r = np.zeros_like(u)
    _load().ref_residual2(_n2(u.shape), _h(u.shape, lengths), u, _ptr(f), r)
    return r


def rbgs2(u, f, nsweeps=1, lengths=(1.0, 1.0)):
    u = _f64(u).copy()
    f = None if f is None else _f64(f)
    _load().ref_rbgs2(_n2(u.shape), _h(u.shape, lengths), u, _ptr(f), nsweeps)
    return u


def restrict2(rf):
    rf = _f64(rf)
    ny, nx = rf.shape
    fc = np.zeros(((ny - 1) // 2 + 1, (nx - 1) // 2 + 1))
    _load().ref_restrict2(_n2(rf.shape), rf, fc)
    return fc


def prolong2(ec, uf):
    ec = _f64(ec)
    uf = _f64(uf).copy()
    _load().ref_prolong2(_n2(ec.shape), ec, uf)
    return uf


def direct2(u, f, lengths=(1.0, 1.0)):
    u = _f64(u).copy()
    f = None if f is None else _f64(f)
    st = _load().ref_direct2(_n2(u.shape), _h(u.shape, lengths), u, _ptr(f))
    if st != OK:
        raise RuntimeError(f"ref_direct2 failed: {st}")
    return u


def mg2(bz0, rtol=1e-10, max_cycles=50, nu1=2, nu2=2, lengths=(1.0, 1.0), P0=None,
        history=False, keep_edges=False):
    """Multigrid solve of (11).  Returns (P0, status, cycles, relres[, hist]).
    With keep_edges, P0's edge values are the Dirichlet data (else zero)."""
    bz0 = _f64(bz0)
    P0 = np.zeros_like(bz0) if P0 is None else _f64(P0).copy()
    cyc = C.c_int(0)
    rel = C.c_double(0.0)
    hist = np.zeros(max_cycles + 1)
    st = _load().ref_mg2_edges(_n2(bz0.shape), _f64(lengths), bz0, P0, rtol, max_cycles, nu1, nu2,
                               C.byref(cyc), C.byref(rel), _ptr(hist), int(keep_edges))
    out = (P0, st, cyc.value, rel.value)
    return out + (hist[: cyc.value + 1],) if history else out


def jacobi2(P1, bz, lengths=(1.0, 1.0)):
    """One step of the paper's lower-boundary Jacobi kernel (Section 4)."""
    P1 = _f64(P1)
    P2 = np.zeros_like(P1)
    _load().ref_jacobi2(_n2(P1.shape), _h(P1.shape, lengths), P1, _f64(bz), P2)
    return P2


def set_threads(n):
    """Threads the oracle's parallel node loops use (OpenMP); returns the
    count in effect.  Results do not depend on it."""
    return _load().ref_set_threads(int(n))


def solve(bz0, xi, alpha, shape, lengths=(1.0, 1.0, 1.0), rtol2=1e-10, rtol3=1e-10,
          max_cycles=100, nu1=2, nu2=2):
    """The three steps of Section 2.2.  Returns (P, status, info dict)."""
    nz, ny, nx = shape
    P = np.zeros(shape)
    info = np.zeros(4)
    st = _load().ref_solve(np.array([nx, ny, nz], dtype=np.int32), _f64(lengths), _f64(bz0),
                           _f64(xi), alpha, P, rtol2, rtol3, max_cycles, nu1, nu2, info)
    return P, st, dict(cycles2d=int(info[0]), cycles3d=int(info[1]),
                       relres2d=float(info[2]), relres3d=float(info[3]))


# ---------------------------------------------------------------- the general operator
def gen_mg(u, a, b, c, rtol=1e-10, max_cycles=50, nu1=2, nu2=2, lengths=(1.0, 1.0, 1.0), planar=False):
    """Multigrid solve of a lap u + b u = c (Section 2.2's general form) in
    place of a copy of u: 3D arrays (nz, ny, nx), or planar (ny, nx) arrays
    for a face (lengths of its two axes).  u's boundary values are the
    Dirichlet data.  rtol < 0 runs exactly max_cycles cycles.  Returns
    (u, status, cycles, relres, hist)."""
    u = _f64(u).copy()
    a, b, c = _f64(a), _f64(b), _f64(c)
    n = _n2(u.shape) if planar else _n3(u.shape)
    if planar:
        n = np.array([n[0], n[1], 1], dtype=np.int32)
    ln = np.asarray(lengths, dtype=np.float64)
    if ln.size < 3:
        ln = np.concatenate([ln, [1.0] * (3 - ln.size)])
    cyc = C.c_int(0)
    rel = C.c_double(0.0)
    hist = np.zeros(max_cycles + 1)
    st = _load().ref_gen_mg(n, ln, 1 if planar else 0, a, b, c, u, float(rtol), int(max_cycles), int(nu1), int(nu2),
                            C.byref(cyc), C.byref(rel), hist.ctypes.data_as(C.c_void_p))
    return u, st, cyc.value, rel.value, hist[: cyc.value + 1]


def gen_levels(shape, lengths=(1.0, 1.0, 1.0), planar=False):
    n = _n2(shape) if planar else _n3(shape)
    if planar:
        n = np.array([n[0], n[1], 1], dtype=np.int32)
    ln = np.asarray(list(lengths) + [1.0] * (3 - len(lengths)), dtype=np.float64)
    return _load().ref_gen_levels(n, ln, 1 if planar else 0)


def gen_residual(u, a, b, c, lengths=(1.0, 1.0, 1.0), planar=False):
    """Residual c/a - (lap_h u + (b/a) u) of the divided form on interior
    nodes (0 elsewhere)."""
    u, a, b, c = _f64(u), _f64(a), _f64(b), _f64(c)
    n = _n2(u.shape) if planar else _n3(u.shape)
    if planar:
        n = np.array([n[0], n[1], 1], dtype=np.int32)
    beta, gamma, r = np.zeros_like(u), np.zeros_like(u), np.zeros_like(u)
    st = _load().ref_gen_normalise(n, 1 if planar else 0, a, b, c, beta, gamma)
    if planar:
        h = np.array([lengths[0] / (u.shape[1] - 1), lengths[1] / (u.shape[0] - 1), 1.0])
    else:
        h = _h(u.shape, lengths)
    _load().ref_gen_residual(n, h, 1 if planar else 0, beta, u, gamma, r)
    return r, st


def _gen_nh(shape, lengths, planar):
    if planar:
        ny, nx = shape
        return (np.array([nx, ny, 1], dtype=np.int32),
                np.array([lengths[0] / (nx - 1), lengths[1] / (ny - 1), 1.0]))
    return _n3(shape), _h(shape, lengths)


def gen_rbgs(u, beta, gamma, nsweeps=1, lengths=(1.0, 1.0, 1.0), planar=False):
    """Red-black Gauss-Seidel sweeps of lap_h u + beta u = gamma on a copy."""
    u = _f64(u).copy()
    n, h = _gen_nh(u.shape, lengths, planar)
    _load().ref_gen_rbgs(n, h, 1 if planar else 0, _f64(beta), u, _f64(gamma), int(nsweeps))
    return u


def gen_direct(u, beta, gamma, lengths=(1.0, 1.0, 1.0), planar=False):
    """Exact solve of lap_h u + beta u = gamma (u's boundary as data)."""
    u = _f64(u).copy()
    n, h = _gen_nh(u.shape, lengths, planar)
    st = _load().ref_gen_direct(n, h, 1 if planar else 0, _f64(beta), u, _f64(gamma))
    return u, st


def gen_inject(beta, kind=0, planar=False):
    """beta on the next coarser grid (kind: STEP_ALL, STEP_XY, STEP_Z)."""
    beta = _f64(beta)
    if planar:
        ny, nx = beta.shape
        n = np.array([nx, ny, 1], dtype=np.int32)
        out = np.zeros(((ny - 1) // 2 + 1, (nx - 1) // 2 + 1))
    else:
        nz, ny, nx = beta.shape
        n = _n3(beta.shape)
        sx = 1 if kind == STEP_Z else 2
        sz = 1 if kind == STEP_XY else 2
        out = np.zeros(((nz - 1) // sz + 1, (ny - 1) // sx + 1, (nx - 1) // sx + 1))
    _load().ref_gen_inject(n, 1 if planar else 0, int(kind), beta, out)
    return out
