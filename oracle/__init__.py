"""Parity oracle for the batched HEALPix spherical harmonic transform.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link or
execute this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.

It wraps ``sht_oracle.c`` (a plain long-double direct-summation implementation of
the transforms defined in Sec. 2.1 and Sec. 2.3 of Tian, Li & Liu,
arXiv:2208.10154) and adds, in plain numpy:

* the conversion between complex (l, m) coefficients and the paper's compact real
  (lmax+1)^2 storage (Appendix A.2, "new storage scheme"), and
* the "traditional" Jacobi iteration of Sec. 4 / Algorithm 2, written in the pixel
  domain: a_0 = A m, a_n = a_{n-1} + A (m - Y a_{n-1}), and the "immediate" mode of
  Algorithm 3 as a Gauss-Seidel sweep over m, and
* the selective (T / E / B) transforms and the pixel-domain E/B separation of
  Sec. 2.3.

Complex coefficient arrays have shape ``[..., lmax+1, lmax+1]`` indexed ``[l, m]``
(m <= l used, m >= 0 only).  Maps are float64 ``[..., 12 nside^2]`` in RING order.

Every function is pinned by tests under ``tests/`` against closed forms, library
routines and brute force; see the test files for which pin covers which function.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sht_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_l = ctypes.POINTER(ctypes.c_long)


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc + OpenMP (IEEE semantics, no fast-math)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_SO)
        L_, I_ = ctypes.c_long, ctypes.c_int
        lib.orc_ring.argtypes = [L_, L_, _d, _d, _l, ctypes.POINTER(I_), _l]
        lib.orc_lambda0.argtypes = [L_, L_, ctypes.c_double, _d]
        lib.orc_lambda_spin.argtypes = [L_, L_, L_, ctypes.c_double, _d]
        lib.orc_alm2map_spin0.argtypes = [L_, L_, L_, _d, _d]
        lib.orc_map2alm_spin0.argtypes = [L_, L_, L_, _d, _d]
        lib.orc_alm2map_spin2.argtypes = [L_, L_, L_, _d, _d, _d, _d]
        lib.orc_map2alm_spin2.argtypes = [L_, L_, L_, _d, _d, _d, _d]
        lib.orc_synth_pixels_spin0.argtypes = [L_, L_, _d, L_, _l, _d]
        lib.orc_synth_pixels_spin2.argtypes = [L_, L_, _d, _d, L_, _l, _d, _d]
        lib.orc_analyze_lm_spin0.argtypes = [L_, L_, _d, L_, _l, _l, _d]
        lib.orc_analyze_lm_spin2.argtypes = [L_, L_, _d, _d, L_, _l, _l, _d, _d]
        lib.orc_alm2map_spin0_strided.argtypes = [L_, L_, L_, _d, _d, L_]
        lib.orc_map2alm_spin0_strided.argtypes = [L_, L_, L_, _d, _d, L_]
        lib.orc_alm2map_spin2_strided.argtypes = [L_, L_, L_, _d, _d, _d, _d, L_]
        lib.orc_map2alm_spin2_strided.argtypes = [L_, L_, L_, _d, _d, _d, _d, L_]
        lib.orc_num_threads.restype = I_
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(_d)


def _pl(a):
    return a.ctypes.data_as(_l)


def num_threads() -> int:
    """OpenMP threads the oracle runs with (OMP_NUM_THREADS or all cores)."""
    return int(_L().orc_num_threads())


def npix(nside: int) -> int:
    return 12 * nside * nside


def ring_info(nside: int) -> dict:
    """Per-ring geometry (rings 1 .. 4 nside - 1): z, sin(theta), pixel count,
    phase shift s (pixel n at phi = pi (2n + s) / N) and first pixel index."""
    nr = 4 * nside - 1
    out = {k: [] for k in ("z", "sth", "n", "s", "first")}
    z, st = ctypes.c_double(), ctypes.c_double()
    n, f = ctypes.c_long(), ctypes.c_long()
    s = ctypes.c_int()
    for i in range(1, nr + 1):
        _L().orc_ring(nside, i, ctypes.byref(z), ctypes.byref(st), ctypes.byref(n), ctypes.byref(s), ctypes.byref(f))
        out["z"].append(z.value); out["sth"].append(st.value); out["n"].append(n.value)
        out["s"].append(s.value); out["first"].append(f.value)
    return {k: np.array(v) for k, v in out.items()}


def pixel_angles(nside: int):
    """(theta, phi) of every pixel centre, RING order."""
    r = ring_info(nside)
    th = np.empty(npix(nside)); ph = np.empty(npix(nside))
    for z, n, s, f in zip(r["z"], r["n"], r["s"], r["first"]):
        th[f:f + n] = np.arccos(z)
        ph[f:f + n] = np.pi * (2 * np.arange(n) + s) / n
    return th, ph


def lambda0(lmax: int, m: int, theta: float) -> np.ndarray:
    out = np.zeros(lmax + 1)
    _L().orc_lambda0(lmax, m, float(theta), _p(out))
    return out


def lambda_spin(lmax: int, m: int, s: int, theta: float) -> np.ndarray:
    out = np.zeros(lmax + 1)
    _L().orc_lambda_spin(lmax, m, s, float(theta), _p(out))
    return out


def _c2r(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a.view(np.float64)


def _tri_mask(lmax):
    l = np.arange(lmax + 1)[:, None]
    m = np.arange(lmax + 1)[None, :]
    return m <= l


# --------------------------------------------------------------------------- transforms
def alm2map(nside: int, lmax: int, alm: np.ndarray) -> np.ndarray:
    """Spin-0 backward transform.  alm: complex [nmaps, L+1, L+1] -> maps [nmaps, Npix]."""
    alm = np.ascontiguousarray(alm * _tri_mask(lmax), dtype=np.complex128)
    k = alm.shape[0]
    out = np.zeros((k, npix(nside)))
    _L().orc_alm2map_spin0(nside, lmax, k, _p(_c2r(alm)), _p(out))
    return out


def map2alm(nside: int, lmax: int, maps: np.ndarray) -> np.ndarray:
    """Spin-0 forward transform.  maps [nmaps, Npix] -> complex [nmaps, L+1, L+1]."""
    maps = np.ascontiguousarray(maps, dtype=np.float64)
    k = maps.shape[0]
    out = np.zeros((k, lmax + 1, lmax + 1), dtype=np.complex128)
    _L().orc_map2alm_spin0(nside, lmax, k, _p(maps), _p(out.view(np.float64)))
    return out


def alm2map_spin2(nside: int, lmax: int, almE: np.ndarray, almB: np.ndarray):
    """Spin-2 backward transform: (E, B) complex [nmaps, L+1, L+1] -> (Q, U) [nmaps, Npix]."""
    m = _tri_mask(lmax)
    almE = np.ascontiguousarray(almE * m, dtype=np.complex128)
    almB = np.ascontiguousarray(almB * m, dtype=np.complex128)
    k = almE.shape[0]
    Q = np.zeros((k, npix(nside))); U = np.zeros((k, npix(nside)))
    _L().orc_alm2map_spin2(nside, lmax, k, _p(_c2r(almE)), _p(_c2r(almB)), _p(Q), _p(U))
    return Q, U


def map2alm_spin2(nside: int, lmax: int, Q: np.ndarray, U: np.ndarray):
    Q = np.ascontiguousarray(Q, dtype=np.float64); U = np.ascontiguousarray(U, dtype=np.float64)
    k = Q.shape[0]
    E = np.zeros((k, lmax + 1, lmax + 1), dtype=np.complex128)
    B = np.zeros_like(E)
    _L().orc_map2alm_spin2(nside, lmax, k, _p(Q), _p(U), _p(E.view(np.float64)), _p(B.view(np.float64)))
    return E, B


def alm2map_iqu(nside: int, lmax: int, alm: np.ndarray) -> np.ndarray:
    """alm complex [nmaps, 3 (T, E, B), L+1, L+1] -> maps [nmaps, 3 (I, Q, U), Npix]."""
    out = np.zeros((alm.shape[0], 3, npix(nside)))
    out[:, 0] = alm2map(nside, lmax, alm[:, 0])
    out[:, 1], out[:, 2] = alm2map_spin2(nside, lmax, alm[:, 1], alm[:, 2])
    return out


def map2alm_iqu(nside: int, lmax: int, maps: np.ndarray) -> np.ndarray:
    out = np.zeros((maps.shape[0], 3, lmax + 1, lmax + 1), dtype=np.complex128)
    out[:, 0] = map2alm(nside, lmax, maps[:, 0])
    out[:, 1], out[:, 2] = map2alm_spin2(nside, lmax, maps[:, 1], maps[:, 2])
    return out


_COMP = {"T": 0, "E": 1, "B": 2}


def _keep(alm: np.ndarray, comps: str) -> np.ndarray:
    """Copy of complex IQU coefficients [n, 3, L+1, L+1] with the components not
    named in comps (letters of "TEB") set to zero: the 0/1 diagonal selector
    lambda^{E,B} of Sec. 2.3, extended by T."""
    out = np.zeros_like(alm)
    for c in comps:
        out[:, _COMP[c]] = alm[:, _COMP[c]]
    return out


def alm2map_sel(nside: int, lmax: int, alm: np.ndarray, comps: str) -> np.ndarray:
    """Backward IQU transform of the named components only (the separate E / B
    transforms of Sec. 3.1): the others' coefficients are treated as zero."""
    return alm2map_iqu(nside, lmax, _keep(alm, comps))


def map2alm_sel(nside: int, lmax: int, maps: np.ndarray, comps: str) -> np.ndarray:
    """Forward IQU transform keeping only the named components (others zero)."""
    return _keep(map2alm_iqu(nside, lmax, maps), comps)


def eb_split(nside: int, lmax: int, maps: np.ndarray):
    """Pixel-domain E/B separation of Sec. 2.3, S^{E,B} = F^t lambda^{E,B} F S:
    analyse the IQU maps, then synthesise once from (T, E) and once from B alone.
    Returns (alm, maps_e, maps_b); maps_e + maps_b = alm2map_iqu(alm)."""
    a = map2alm_iqu(nside, lmax, maps)
    return a, alm2map_iqu(nside, lmax, _keep(a, "TE")), alm2map_iqu(nside, lmax, _keep(a, "B"))


def synth(nside, lmax, alm, pol):
    return alm2map_iqu(nside, lmax, alm) if pol else alm2map(nside, lmax, alm)


def analyse(nside, lmax, maps, pol):
    return map2alm_iqu(nside, lmax, maps) if pol else map2alm(nside, lmax, maps)


def map2alm_iter(nside: int, lmax: int, maps: np.ndarray, niter: int, pol: bool = False):
    """Sec. 4, Algorithm 2 ("traditional" iteration): alm updated outside the
    m-loop, Jacobi form.  Returns (alm, residual_norms) where residual_norms[n] is
    ||m - Y a_n||_2 over all pixels of all maps (n = 0 .. niter)."""
    a = analyse(nside, lmax, maps, pol)
    res = []
    for it in range(niter + 1):
        r = maps - synth(nside, lmax, a, pol)
        res.append(float(np.sqrt(np.sum(r * r))))
        if it == niter:
            break
        a = a + analyse(nside, lmax, r, pol)
    return a, np.array(res)


def map2alm_immediate(nside: int, lmax: int, maps: np.ndarray, niter: int, pol: bool = False):
    """Sec. 4, Algorithm 3 ("immediate" iteration): the coefficients of each m are
    updated inside the m-loop, so every later m already sees them.  Read as a
    Gauss-Seidel sweep over m in increasing order, in the pixel domain: start from
    a = A m and the residual r = m - Y a; then, per sweep and per m = 0 .. lmax,
    take the order-m part of A r as the update of a_m and subtract its synthesis
    from r at once.  Returns (alm, residual_norms) as map2alm_iter does
    (residual_norms[n] = ||r||_2 after sweep n, n = 0 .. niter)."""
    a = analyse(nside, lmax, maps, pol)
    r = maps - synth(nside, lmax, a, pol)
    res = [float(np.sqrt(np.sum(r * r)))]
    for _ in range(niter):
        for m in range(lmax + 1):
            d = analyse(nside, lmax, r, pol)
            da = np.zeros_like(d)
            da[..., :, m] = d[..., :, m]
            a = a + da
            r = r - synth(nside, lmax, da, pol)
        res.append(float(np.sqrt(np.sum(r * r))))
    return a, np.array(res)


def timing_sample_iqu(nside: int, lmax: int, alm1: np.ndarray, maps1: np.ndarray, stride: int):
    """Run the oracle's IQU alm2map on every `stride`-th ring and its map2alm on
    every `stride`-th m, for ONE map triple (alm1 complex [3, L+1, L+1], maps1
    [3, Npix]).  Returns (seconds_alm2map, seconds_map2alm) of the sample; the
    full transforms visit stride times as many rings / m values."""
    import time
    L = lmax
    msk = _tri_mask(L)
    a = [np.ascontiguousarray(alm1[c][None] * msk, dtype=np.complex128) for c in range(3)]
    out = np.zeros((3, 1, npix(nside)))
    t0 = time.perf_counter()
    _L().orc_alm2map_spin0_strided(nside, L, 1, _p(_c2r(a[0])), _p(out[0]), stride)
    _L().orc_alm2map_spin2_strided(nside, L, 1, _p(_c2r(a[1])), _p(_c2r(a[2])), _p(out[1]), _p(out[2]), stride)
    t1 = time.perf_counter()
    mp = [np.ascontiguousarray(maps1[c][None], dtype=np.float64) for c in range(3)]
    r = np.zeros((3, 1, L + 1, L + 1), dtype=np.complex128)
    _L().orc_map2alm_spin0_strided(nside, L, 1, _p(mp[0]), _p(r[0].view(np.float64)), stride)
    _L().orc_map2alm_spin2_strided(nside, L, 1, _p(mp[1]), _p(mp[2]), _p(r[1].view(np.float64)),
                                   _p(r[2].view(np.float64)), stride)
    t2 = time.perf_counter()
    return t1 - t0, t2 - t1


# --------------------------------------------------------------------------- sampled
def synth_pixels(nside: int, lmax: int, alm1: np.ndarray, pix, pol: bool = False):
    """Map values of ONE map at selected pixels.  alm1: complex [L+1, L+1] (spin 0)
    or [3, L+1, L+1] (T, E, B).  Returns [npts] or [3, npts]."""
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    msk = _tri_mask(lmax)
    if not pol:
        out = np.zeros(len(pix))
        a = np.ascontiguousarray(alm1 * msk, dtype=np.complex128)
        _L().orc_synth_pixels_spin0(nside, lmax, _p(_c2r(a)), len(pix), _pl(pix), _p(out))
        return out
    out = np.zeros((3, len(pix)))
    out[0] = synth_pixels(nside, lmax, alm1[0], pix, False)
    aE = np.ascontiguousarray(alm1[1] * msk, dtype=np.complex128)
    aB = np.ascontiguousarray(alm1[2] * msk, dtype=np.complex128)
    q = np.zeros(len(pix)); u = np.zeros(len(pix))
    _L().orc_synth_pixels_spin2(nside, lmax, _p(_c2r(aE)), _p(_c2r(aB)), len(pix), _pl(pix), _p(q), _p(u))
    out[1], out[2] = q, u
    return out


def analyze_lm(nside: int, lmax: int, map1: np.ndarray, ls, ms, pol: bool = False):
    """a_lm of ONE map at selected (l, m).  map1: [Npix] or [3, Npix].
    Returns complex [npts] or [3, npts]."""
    ls = np.ascontiguousarray(ls, dtype=np.int64); ms = np.ascontiguousarray(ms, dtype=np.int64)
    if not pol:
        out = np.zeros(len(ls), dtype=np.complex128)
        mp = np.ascontiguousarray(map1, dtype=np.float64)
        _L().orc_analyze_lm_spin0(nside, lmax, _p(mp), len(ls), _pl(ls), _pl(ms), _p(out.view(np.float64)))
        return out
    out = np.zeros((3, len(ls)), dtype=np.complex128)
    out[0] = analyze_lm(nside, lmax, map1[0], ls, ms, False)
    q = np.ascontiguousarray(map1[1], dtype=np.float64); u = np.ascontiguousarray(map1[2], dtype=np.float64)
    e = np.zeros(len(ls), dtype=np.complex128); b = np.zeros(len(ls), dtype=np.complex128)
    _L().orc_analyze_lm_spin2(nside, lmax, _p(q), _p(u), len(ls), _pl(ls), _pl(ms),
                              _p(e.view(np.float64)), _p(b.view(np.float64)))
    out[1], out[2] = e, b
    return out


# --------------------------------------------------------------------------- compact storage
def _compact_index(L: int):
    """Flat compact positions of Re a_lm (all l >= m) and Im a_lm (m >= 1), in the
    order of the (l, m) lists returned: Re at (row l, col m), Im at
    (row l-m, col L+1-m); flat index col*(L+1) + row (Appendix A.2)."""
    l, m = np.tril_indices(L + 1)
    re = m * (L + 1) + l
    sel = m >= 1
    im = (L + 1 - m[sel]) * (L + 1) + (l[sel] - m[sel])
    return l, m, re, sel, im


def to_compact(alm: np.ndarray) -> np.ndarray:
    """Complex [..., L+1, L+1] -> the paper's compact real (L+1)x(L+1) matrix
    (Appendix A.2): Re a_lm at (row l, col m); Im a_lm (m >= 1) at
    (row l - m, col L + 1 - m).  0-based, stored column-major: flat index
    col * (L+1) + row."""
    L = alm.shape[-1] - 1
    l, m, re, sel, im = _compact_index(L)
    out = np.zeros(alm.shape[:-2] + ((L + 1) * (L + 1),))
    vals = alm[..., l, m]
    out[..., re] = vals.real
    out[..., im] = vals[..., sel].imag
    return out


def from_compact(c: np.ndarray, lmax: int) -> np.ndarray:
    L = lmax
    l, m, re, sel, im = _compact_index(L)
    out = np.zeros(c.shape[:-1] + (L + 1, L + 1), dtype=np.complex128)
    vals = c[..., re].astype(np.complex128)
    vals[..., sel] += 1j * c[..., im]
    out[..., l, m] = vals
    return out
