"""Statistics of a bubble (or droplet) swarm, as in the paper's swarm section:
the PDF of the interfacial mean curvature kappa = div n (Eq. kappa_radius,
kappa = 2/R on a sphere), the PDF of the equivalent diameter of the dispersed
components, and the isotropic kinetic-energy spectrum E(k) of the carrier-phase
velocity fluctuations.

The curvature histogram and the component volumes are computed on the device
(lbm_curvature_histogram, lbm_component_volumes); the spectrum is host
post-processing of the velocity field (one FFT per component), as the paper's
spectrum is post-processing of its fields.
"""
from __future__ import annotations

import math

import numpy as np

from . import lbm as L

DEFAULT_Q_BAND = 3.0 / 16.0     # interface cells: phi in [1/4, 3/4]


def curvature_pdf(lat: L.Lattice, kmin: float, kmax: float, nbins: int = 64,
                  q_band: float = DEFAULT_Q_BAND):
    """(bin centres, PDF over [kmin, kmax), counts incl. the two overflow bins)."""
    counts = lat.curvature_histogram(q_band, kmin, kmax, nbins)
    width = (kmax - kmin) / nbins
    centres = kmin + width * (np.arange(nbins) + 0.5)
    inside = counts[1:-1].astype(np.float64)
    tot = inside.sum()
    pdf = inside / (tot * width) if tot > 0 else inside
    return centres, pdf, counts


def equivalent_diameters(lat: L.Lattice) -> np.ndarray:
    """D_eq of every dispersed component from its cell count V: (6 V / pi)^(1/3) in 3D,
    (4 V / pi)^(1/2) in 2D; largest first."""
    v = lat.component_volumes().astype(np.float64)
    if lat.params.dim == 3:
        return np.cbrt(6.0 * v / math.pi)
    return np.sqrt(4.0 * v / math.pi)


def energy_spectrum(u: np.ndarray, carrier: np.ndarray | None = None):
    """Isotropic kinetic-energy spectrum of the velocity fluctuations.

    u: (dim,) + shape velocity field (arrays [z][y][x] or [y][x]) of a periodic
    cubic (square) box of edge n; carrier: optional weight (e.g. the liquid
    indicator) applied to the fluctuations u - <u>_carrier.  With û the discrete
    Fourier transform normalised by the cell count, E(k) = sum over wavevectors
    with round(|k|) = k of (1/2) |û|^2, k in units of 2 pi / n, so that
    sum_k E(k) = (1/2) <|u'|^2> (Parseval).  Returns (k, E) over every shell present,
    k = 0 .. round(sqrt(dim) n / 2); shells above n / 2 are only partly filled."""
    u = np.asarray(u, dtype=np.float64)
    dim = u.shape[0]
    shape = u.shape[1:]
    n = shape[0]
    if any(s != n for s in shape):
        raise ValueError("energy_spectrum needs a cubic (square) box")
    if carrier is None:
        w = np.ones(shape)
        mean = u.reshape(dim, -1).mean(axis=1)
    else:
        w = np.asarray(carrier, dtype=np.float64)
        mean = (u * w).reshape(dim, -1).sum(axis=1) / max(w.sum(), 1e-300)
    freqs = np.fft.fftfreq(n) * n
    grids = np.meshgrid(*([freqs] * dim), indexing="ij")
    kmag = np.sqrt(sum(g * g for g in grids))
    shell = np.rint(kmag).astype(np.int64)
    kmax = int(shell.max())
    E = np.zeros(kmax + 1)
    cells = float(np.prod(shape))
    for a in range(dim):
        f = np.fft.fftn((u[a] - mean[a]) * w) / cells
        e = 0.5 * (f.real ** 2 + f.imag ** 2)
        E += np.bincount(shell.ravel(), weights=e.ravel(), minlength=kmax + 1)
    return np.arange(kmax + 1), E
