"""Synthetic lower-boundary magnetograms Bz0(x, y).

The paper drives every example with Gaussian flux sources of the form
B0 * exp(-r^2 / l^2) on the lower boundary (Section 3.1).  The benchmark
workloads use the same source shape, arranged as bipoles with exactly zero
net flux over the interior nodes.

Arrays are float64 with shape (ny, nx): x varies fastest, node (i, j) sits at
x = x0 + i*lx/(nx-1), y = y0 + j*ly/(ny-1).  Edge nodes are set to zero
because the boundary potential vanishes on the side walls and Bz0 on the
edges is never read by the solve.
"""

from __future__ import annotations

import numpy as np


def _nodes(n: int, length: float, origin: float) -> np.ndarray:
    return origin + np.arange(n, dtype=np.float64) * (length / (n - 1))


def gaussian_sources(nx, ny, lx, ly, sources, width, x0=0.0, y0=0.0):
    """Sum of Gaussian sources B0*exp(-r^2/l^2) (Section 3.1).

    sources: iterable of (xc, yc, B0) in physical coordinates.
    width:   the source width l (shared by all sources).
    Edge nodes are zeroed.
    """
    x = _nodes(nx, lx, x0)[None, :]
    y = _nodes(ny, ly, y0)[:, None]
    bz = np.zeros((ny, nx), dtype=np.float64)
    for xc, yc, amp in sources:
        bz += amp * np.exp(-((x - xc) ** 2 + (y - yc) ** 2) / (width * width))
    _zero_edges(bz)
    return bz


def _zero_edges(a: np.ndarray) -> None:
    a[0, :] = 0.0
    a[-1, :] = 0.0
    a[:, 0] = 0.0
    a[:, -1] = 0.0


def bipolar_magnetogram(nx, ny, lx, ly, nbip, rng, sigma=None,
                        sigma_range=(0.03, 0.1), noise_frac=0.0):
    """Seeded bipolar magnetogram with exactly zero net interior flux.

    For each bipole, in this order, the generator draws the positive centre
    (2 uniforms), the negative centre (2 uniforms) and, when ``sigma`` is
    None, a width from U[sigma_range).  Centres are uniform in
    [0.2, 0.8]^2 in units of (lx, ly).  Each source is exp(-r^2/sigma^2)
    with amplitude +1 or -1.  The negative part is rescaled by S+/S- (sums
    over interior nodes) so the interior flux is zero to rounding.  With
    ``noise_frac`` > 0, Gaussian noise of standard deviation
    noise_frac*max|Bz0| is added to interior nodes and the interior mean is
    removed afterwards.
    """
    x = _nodes(nx, lx, 0.0)[None, :]
    y = _nodes(ny, ly, 0.0)[:, None]
    pos = np.zeros((ny, nx), dtype=np.float64)
    neg = np.zeros((ny, nx), dtype=np.float64)
    for _ in range(nbip):
        cp = rng.uniform(0.2, 0.8, size=2)
        cn = rng.uniform(0.2, 0.8, size=2)
        s = float(sigma) if sigma is not None else float(rng.uniform(*sigma_range))
        pos += np.exp(-((x - cp[0] * lx) ** 2 + (y - cp[1] * ly) ** 2) / (s * s))
        neg += np.exp(-((x - cn[0] * lx) ** 2 + (y - cn[1] * ly) ** 2) / (s * s))
    inner = (slice(1, -1), slice(1, -1))
    s_pos = pos[inner].sum()
    s_neg = neg[inner].sum()
    bz = pos - (s_pos / s_neg) * neg
    if noise_frac > 0.0:
        amp = noise_frac * np.abs(bz[inner]).max()
        noise = rng.normal(0.0, amp, size=(ny - 2, nx - 2))
        bz[inner] += noise
        bz[inner] -= bz[inner].mean()
    _zero_edges(bz)
    return bz


def fourier_mode(nx, ny, lx, ly, m, n, amp=1.0):
    """amp * sin(m*pi*x/lx) * sin(n*pi*y/ly) sampled on the nodes.

    A single Fourier mode vanishes on every edge, so it satisfies the side
    boundary condition of the lower-boundary problem exactly.
    """
    x = _nodes(nx, lx, 0.0)[None, :]
    y = _nodes(ny, ly, 0.0)[:, None]
    bz = amp * np.sin(m * np.pi * x / lx) * np.sin(n * np.pi * y / ly)
    _zero_edges(bz)
    return bz
