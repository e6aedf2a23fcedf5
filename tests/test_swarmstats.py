"""Host-side spectrum of the swarm statistics (paper_2603_17481_amd.swarmstats):
Parseval, a single Fourier mode, the carrier weighting."""
import numpy as np

from paper_2603_17481_amd import swarmstats as S


def test_spectrum_parseval_and_single_mode():
    rng = np.random.default_rng(3)
    n = 32
    u = rng.normal(size=(3, n, n, n))
    k, E = S.energy_spectrum(u)
    up = u - u.reshape(3, -1).mean(axis=1)[:, None, None, None]
    assert abs(E.sum() - 0.5 * (up ** 2).sum(axis=0).mean()) < 1e-12 * E.sum()
    assert E[0] < 1e-25   # the mean is removed
    # one mode along x of wavenumber 5, amplitude 0.3 in u_y: energy (1/2)(0.3^2 / 2) at k = 5
    x = np.arange(n)[None, None, :] * np.ones((n, n, n))
    v = np.zeros((3, n, n, n))
    v[1] = 0.3 * np.sin(2 * np.pi * 5 * x / n)
    k, E = S.energy_spectrum(v)
    assert abs(E[5] - 0.5 * 0.3 ** 2 / 2) < 1e-15 and abs(E.sum() - E[5]) < 1e-15
    # the same mode along z lands in the same shell; a diagonal mode (3, 4, 0) in shell 5
    z = np.arange(n)[:, None, None] * np.ones((n, n, n))
    y = np.arange(n)[None, :, None] * np.ones((n, n, n))
    v2 = np.zeros((3, n, n, n))
    v2[0] = 0.3 * np.sin(2 * np.pi * 5 * z / n)
    v2[2] = 0.3 * np.cos(2 * np.pi * (3 * x + 4 * y) / n)
    k, E2 = S.energy_spectrum(v2)
    assert abs(E2[5] - 2 * 0.5 * 0.3 ** 2 / 2) < 1e-15


def test_spectrum_carrier_weighting_2d():
    rng = np.random.default_rng(4)
    n = 64
    u = rng.normal(size=(2, n, n))
    w = (rng.uniform(size=(n, n)) > 0.3).astype(float)
    k, E = S.energy_spectrum(u, carrier=w)
    mean = (u * w).reshape(2, -1).sum(axis=1) / w.sum()
    up = (u - mean[:, None, None]) * w
    assert abs(E.sum() - 0.5 * (up ** 2).sum(axis=0).mean()) < 1e-12 * E.sum()
