"""Literal per-pixel spherical-harmonic sums for tiny HEALPix maps.

These are the brute-force pins of the oracle: every pixel, every (l, m) with
m = -l .. l, the harmonic evaluated from an independent source (scipy's
``sph_harm_y`` for spin 0, the explicit Goldberg et al. (1967) sum for spin 2).
No recursion, no ring grouping, no reality-condition shortcut.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import sph_harm_y


def healpix_centres(nside: int):
    """Pixel centres straight from the HEALPix definition (Gorski et al. 2005),
    written independently of the oracle's ring routine: loops over pixels."""
    ns = nside
    th, ph = [], []
    for i in range(1, 4 * ns):
        if i < ns:
            z, n, s = 1 - i * i / (3 * ns * ns), 4 * i, 1
        elif i > 3 * ns:
            j = 4 * ns - i
            z, n, s = -(1 - j * j / (3 * ns * ns)), 4 * j, 1
        else:
            z, n, s = (4 * ns - 2 * i) / (3 * ns), 4 * ns, 1 if (i - ns) % 2 == 0 else 0
        for k in range(n):
            th.append(math.acos(z))
            ph.append(math.pi * (2 * k + s) / n)
    return np.array(th), np.array(ph)


def full_m(alm: np.ndarray):
    """Extend m >= 0 coefficients of a real field to m = -l .. l: a_{l,-m} = (-1)^m conj(a_lm)."""
    L = alm.shape[-1] - 1
    out = {}
    for l in range(L + 1):
        for m in range(0, l + 1):
            out[(l, m)] = alm[l, m]
            if m > 0:
                out[(l, -m)] = (-1) ** m * np.conj(alm[l, m])
    return out


def y_lm(l, m, th, ph):
    return sph_harm_y(l, m, th, ph)


def goldberg(s, l, m, th, ph):
    """{}_sY_lm by the explicit finite sum of Goldberg et al. (1967)."""
    if l < abs(s) or l < abs(m):
        return np.zeros_like(th, dtype=complex)
    pre = (-1) ** m * math.sqrt(math.factorial(l + m) * math.factorial(l - m) * (2 * l + 1)
                                / (4 * math.pi * math.factorial(l + s) * math.factorial(l - s)))
    tot = np.zeros_like(th, dtype=complex)
    for r in range(0, l - s + 1):
        k2 = r + s - m
        if k2 < 0 or k2 > l + s:
            continue
        c = math.comb(l - s, r) * math.comb(l + s, k2) * (-1) ** (l - r - s)
        # sin^{2l}(th/2) cot^{2r+s-m}(th/2) = sin^{2l-p} cos^{p}, p = 2r+s-m
        p = 2 * r + s - m
        tot = tot + c * np.sin(th / 2) ** (2 * l - p) * np.cos(th / 2) ** p
    return pre * tot * np.exp(1j * m * ph)


def synth0(nside, alm):
    th, ph = healpix_centres(nside)
    T = np.zeros(len(th), dtype=complex)
    for (l, m), a in full_m(alm).items():
        T += a * y_lm(l, m, th, ph)
    return T


def anal0(nside, maps, lmax):
    th, ph = healpix_centres(nside)
    dsig = 4 * math.pi / len(th)
    out = np.zeros((lmax + 1, lmax + 1), dtype=complex)
    for l in range(lmax + 1):
        for m in range(l + 1):
            out[l, m] = dsig * np.sum(maps * np.conj(y_lm(l, m, th, ph)))
    return out


def synth2(nside, almE, almB):
    th, ph = healpix_centres(nside)
    P = np.zeros(len(th), dtype=complex)
    E, B = full_m(almE), full_m(almB)
    for key in E:
        l, m = key
        a2 = -(E[key] + 1j * B[key])
        P += a2 * goldberg(2, l, m, th, ph)
    return P.real, P.imag


def anal2(nside, Q, U, lmax):
    th, ph = healpix_centres(nside)
    dsig = 4 * math.pi / len(th)
    E = np.zeros((lmax + 1, lmax + 1), dtype=complex)
    B = np.zeros_like(E)
    for l in range(2, lmax + 1):
        for m in range(l + 1):
            a2 = dsig * np.sum((Q + 1j * U) * np.conj(goldberg(2, l, m, th, ph)))
            am = dsig * np.sum((Q - 1j * U) * np.conj(goldberg(-2, l, m, th, ph)))
            E[l, m] = -(a2 + am) / 2
            B[l, m] = 1j * (a2 - am) / 2
    return E, B
