"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds only random-number recipes: no part of the transform.  Every
map is drawn from its own stream, ``SeedSequence([220810154, workload, index])``,
so a map is the same whatever batch it is generated in (the serving tests rely
on that).

Recipe (a stand-in for the paper's Planck-spectrum simulations, which are not
available):

* spin 0: a_l0 = sqrt(C_l) g (real), a_lm = sqrt(C_l/2) (g1 + i g2) for m > 0,
  with C_l = 1/(l+1)^2 for l >= 2 and a_00 = a_1m = 0;
* IQU: a_T = sqrt(C_TT) z1, a_E = sqrt(C_EE) (rho z1 + sqrt(1-rho^2) z2),
  a_B = sqrt(C_BB) z3, C_EE = 0.1 C_TT, C_BB = 0.01 C_TT, rho = 0.5
  (TE correlation coefficient);
* pixel noise: white Gaussian with sigma = f * RMS of each map component.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 220810154


def rng(workload: int, index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, int(workload), int(index)])))


def cl_tt(lmax: int) -> np.ndarray:
    l = np.arange(lmax + 1, dtype=np.float64)
    c = 1.0 / (l + 1.0) ** 2
    c[:2] = 0.0
    return c


def _gauss_lm(g: np.random.Generator, lmax: int, n: int) -> np.ndarray:
    """n independent unit-variance complex Gaussian (l, m) fields, [n, L+1, L+1]:
    real N(0,1) at m = 0, (N(0,1) + i N(0,1))/sqrt(2) at m > 0, zero for m > l."""
    L = lmax
    z = g.standard_normal((n, L + 1, L + 1, 2))
    out = (z[..., 0] + 1j * z[..., 1]) / np.sqrt(2.0)
    out[:, :, 0] = z[:, :, 0, 0]
    l = np.arange(L + 1)[:, None]
    m = np.arange(L + 1)[None, :]
    return np.where(m <= l, out, 0.0)


def gaussian_alm(lmax: int, nmaps: int, pol: bool, workload: int, first: int = 0) -> np.ndarray:
    """Complex coefficients, [nmaps, L+1, L+1] (spin 0) or [nmaps, 3, L+1, L+1] (T, E, B)."""
    L = lmax
    s = np.sqrt(cl_tt(L))[:, None]
    if not pol:
        out = np.zeros((nmaps, L + 1, L + 1), dtype=np.complex128)
        for k in range(nmaps):
            out[k] = s * _gauss_lm(rng(workload, first + k), L, 1)[0]
        return out
    out = np.zeros((nmaps, 3, L + 1, L + 1), dtype=np.complex128)
    rho = 0.5
    for k in range(nmaps):
        z = _gauss_lm(rng(workload, first + k), L, 3)
        out[k, 0] = s * z[0]
        out[k, 1] = np.sqrt(0.1) * s * (rho * z[0] + np.sqrt(1.0 - rho * rho) * z[1])
        out[k, 2] = np.sqrt(0.01) * s * z[2]
    return out


def white_noise_like(maps: np.ndarray, frac: float, workload: int, first: int = 0) -> np.ndarray:
    """White Gaussian pixel noise, sigma = frac * RMS of each map component."""
    out = np.empty_like(maps)
    for k in range(maps.shape[0]):
        g = rng(workload + 1000, first + k)
        rms = np.sqrt(np.mean(maps[k] ** 2, axis=-1, keepdims=True))
        out[k] = frac * rms * g.standard_normal(maps[k].shape)
    return out


def white_maps(npix: int, nmaps: int, ncomp: int, workload: int, first: int = 0) -> np.ndarray:
    """Unit-variance white Gaussian maps [nmaps, ncomp, npix] (not band limited)."""
    out = np.empty((nmaps, ncomp, npix))
    for k in range(nmaps):
        out[k] = rng(workload + 2000, first + k).standard_normal((ncomp, npix))
    return out
