"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package only draws and evaluates *inputs*: boundary magnetograms Bz0,
the cross-field profile xi(z) and its derivative, the background atmosphere
p_b(z), rho_b(z), the request stream of the serving workload, and the
coefficients and data of the general problem a lap u + b u = c.  It holds
none of the solver's arithmetic (no discrete operator, no multigrid, no field
recovery), so either side may import it without sharing method code.
"""

from .magnetogram import bipolar_magnetogram, gaussian_sources, fourier_mode
from .workloads import (
    Grid,
    Model,
    Workload,
    make_grid,
    xi_exponential,
    isothermal_background,
    make_model,
    workload,
    serving_requests,
    request_workload,
    nruns,
    SERVING_SHAPES,
    WORKLOAD_NAMES,
)
from . import paper
from .paper import paper_workload
from .general import general_problem

__all__ = [
    "bipolar_magnetogram",
    "gaussian_sources",
    "fourier_mode",
    "Grid",
    "Model",
    "Workload",
    "make_grid",
    "xi_exponential",
    "isothermal_background",
    "make_model",
    "workload",
    "serving_requests",
    "request_workload",
    "nruns",
    "SERVING_SHAPES",
    "WORKLOAD_NAMES",
    "paper",
    "paper_workload",
    "general_problem",
]
