"""Named synthetic workloads and the model profiles they use.

A workload fixes a grid, the model parameters (alpha, xi(z), background
atmosphere, mu0, g) and a seeded boundary magnetogram.  The cross-field
profile has the exponential form used by the paper's xi_1 example
(Section 3.2): xi(z) = a*exp(-z/h), with the analytic derivative
xi'(z) = -(a/h)*exp(-z/h).

Units: the benchmark workloads live on the unit box in arbitrary units with
mu0 = 1 and g = 1, and an isothermal background p_b = rho_b = exp(-g z).
That background satisfies hydrostatic balance p_b' = -rho_b g, which the
force-balance check of equation (1) needs.

The grid is vertex-centred with n = 2^L + 1 nodes per axis.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .magnetogram import bipolar_magnetogram


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int
    lx: float = 1.0
    ly: float = 1.0
    lz: float = 1.0

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def spacing(self):
        return (self.lx / (self.nx - 1), self.ly / (self.ny - 1), self.lz / (self.nz - 1))

    @property
    def npoints(self):
        return self.nx * self.ny * self.nz

    def z(self):
        return np.arange(self.nz, dtype=np.float64) * (self.lz / (self.nz - 1))


@dataclass
class Model:
    alpha: float
    xi: np.ndarray
    dxi: np.ndarray
    pb: np.ndarray
    rhob: np.ndarray
    mu0: float = 1.0
    g: float = 1.0


def make_grid(nx, ny=None, nz=None, lx=1.0, ly=1.0, lz=1.0) -> Grid:
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return Grid(int(nx), int(ny), int(nz), float(lx), float(ly), float(lz))


def xi_exponential(z, a, h):
    """xi(z) = a*exp(-z/h) and xi'(z) = -(a/h)*exp(-z/h)."""
    e = np.exp(-np.asarray(z, dtype=np.float64) / h)
    return a * e, -(a / h) * e


def isothermal_background(z, g=1.0):
    """p_b = rho_b = exp(-g z): unit temperature, p_b' = -rho_b g."""
    p = np.exp(-g * np.asarray(z, dtype=np.float64))
    return p, p.copy()


def make_model(grid: Grid, alpha, a, h, mu0=1.0, g=1.0) -> Model:
    z = grid.z()
    xi, dxi = xi_exponential(z, a, h)
    pb, rhob = isothermal_background(z, g)
    return Model(float(alpha), xi, dxi, pb, rhob, float(mu0), float(g))


@dataclass
class Workload:
    name: str
    grid: Grid
    model: Model
    bz0: np.ndarray
    seed: int
    target_error: float
    params: dict = field(default_factory=dict)


# name -> (grid dims, list of (alpha, a, h, seed)), bipole recipe, error target
_SPECS = {
    # potential field, FP64, V(2,2) to relative residual 1e-10
    "potential-33": dict(dims=(33, 33, 33), runs=[(0.0, 0.0, 0.2, 1)],
                         nbip=2, sigma=0.08, noise=0.0, target=1e-10),
    # linear MHS, FP64 to 1e-10, then fields
    "mhs-129": dict(dims=(129, 129, 129), runs=[(0.5, 0.5, 0.2, 2)],
                    nbip=6, sigma=None, noise=0.0, target=1e-10),
    # the headline size: alpha in {0, 0.5, 1} x a in {0, 0.5}, seeds 31..36
    "mhs-257": dict(dims=(257, 257, 257),
                    runs=[(al, a, 0.2, 31 + 2 * ia + ja)
                          for ia, al in enumerate((0.0, 0.5, 1.0))
                          for ja, a in enumerate((0.0, 0.5))],
                    nbip=6, sigma=None, noise=0.0, target=1e-8),
    # large single equilibrium, dz = 2 dx on the unit box
    "mhs-513x513x257": dict(dims=(513, 513, 257), runs=[(0.8, 1.0, 0.1, 4)],
                            nbip=40, sigma=None, noise=0.01, target=1e-8),
}

WORKLOAD_NAMES = tuple(_SPECS)


def workload(name: str, run: int = 0, dims=None) -> Workload:
    """Build a named workload.  ``dims`` overrides the grid (same recipe)."""
    spec = _SPECS[name]
    nx, ny, nz = spec["dims"] if dims is None else dims
    alpha, a, h, seed = spec["runs"][run]
    grid = make_grid(nx, ny, nz)
    rng = np.random.default_rng(seed)
    bz0 = bipolar_magnetogram(nx, ny, grid.lx, grid.ly, spec["nbip"], rng,
                              sigma=spec["sigma"], noise_frac=spec["noise"])
    model = make_model(grid, alpha, a, h)
    return Workload(name, grid, model, bz0, seed, spec["target"],
                    dict(alpha=alpha, a=a, h=h, run=run))


def nruns(name: str) -> int:
    return len(_SPECS[name]["runs"])


SERVING_SHAPES = ((65, 65, 65), (129, 129, 129), (129, 129, 65), (257, 257, 257))


def serving_requests(n=512, arrival_seed=7, first_seed=1000, shapes=SERVING_SHAPES):
    """The serving stream: per-request parameters and unit-rate arrival gaps.

    Request i uses seed first_seed+i for everything it draws: its shape
    (uniform over ``shapes``), alpha ~ U[0,1), a ~ U[0,1], h = 0.2, the
    number of bipoles ~ U{4..20} and the bipoles themselves
    (sigma ~ U[0.03, 0.1]).  Arrival gaps are Exp(1) draws from
    ``arrival_seed``; the caller scales them by 1/rate.
    Returns a list of dicts; the magnetogram is built lazily by
    ``request_workload``.
    """
    arr = np.random.default_rng(arrival_seed).exponential(1.0, size=n)
    out = []
    t = 0.0
    for i in range(n):
        rng = np.random.default_rng(first_seed + i)
        shape, alpha, a, nbip = _draw_request_params(rng, shapes)
        t += float(arr[i])
        out.append(dict(id=i, seed=first_seed + i, dims=shape, alpha=alpha, a=a,
                        h=0.2, nbip=nbip, arrival_unit=t, shapes=tuple(shapes)))
    return out


def _draw_request_params(rng, shapes):
    shape = tuple(shapes[int(rng.integers(0, len(shapes)))])
    alpha = float(rng.uniform(0.0, 1.0))
    a = float(rng.uniform(0.0, 1.0))
    nbip = int(rng.integers(4, 21))
    return shape, alpha, a, nbip


def request_workload(req: dict) -> Workload:
    """Materialise one serving request (grid, model, magnetogram)."""
    nx, ny, nz = req["dims"]
    grid = make_grid(nx, ny, nz)
    rng = np.random.default_rng(req["seed"])
    # replay the draws that chose shape/alpha/a/nbip so the bipoles come after
    _draw_request_params(rng, req.get("shapes", SERVING_SHAPES))
    bz0 = bipolar_magnetogram(nx, ny, grid.lx, grid.ly, req["nbip"], rng, sigma=None)
    model = make_model(grid, req["alpha"], req["a"], req["h"])
    return Workload(f"serve-{req['id']}", grid, model, bz0, req["seed"], 1e-8,
                    dict(alpha=req["alpha"], a=req["a"], h=req["h"]))
