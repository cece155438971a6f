"""ctypes binding of libsht (include/sht.h): argument marshalling only.

Device buffers are torch tensors on the plan's GPU; every transform step runs in
the library's HIP kernels.  If the library has not been built this module
raises on first use; there is no fallback implementation.

Layouts (see include/sht.h): maps float64 [nmaps, ncomp, 12 nside^2] (RING
order), alm float64 [nmaps, ncomp, (lmax+1)^2] in the compact real storage of
the paper's Appendix A.2, ncomp = 1 (spin 0) or 3 (spin 2: T, E, B / I, Q, U).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsht.so")

SHT_OK, SHT_ERR_ARG, SHT_ERR_NOMEM, SHT_ERR_DEVICE, SHT_ERR_UNSUPPORTED = 0, -1, -2, -3, -4
SHT_FP64, SHT_FP32, SHT_BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": SHT_FP64, "fp32": SHT_FP32, "bf16x3": SHT_BF16X3}

EXPORTS = ["sht_plan_create", "sht_plan_destroy", "sht_plan_set_precision", "sht_plan_set_stream",
           "sht_plan_set_nmaps", "sht_plan_set_chunk", "sht_plan_workspace_bytes", "sht_plan_table_bytes",
           "sht_plan_set_workspace", "sht_alm2map", "sht_map2alm", "sht_map2alm_iter", "sht_plan_sync",
           "sht_last_error", "sht_plan_set_profiling", "sht_plan_get_profile", "sht_alm2map_sel",
           "sht_map2alm_sel", "sht_eb_split", "sht_map2alm_immediate", "sht_plan_ring_rows",
           "sht_alm2map_noalloc", "sht_plan_create_part"]

STAGES = ["fft_fwd", "fft_inv", "residual", "m2a_spin0", "m2a_spin2", "a2m_spin0", "a2m_spin2", "alm_layout"]

_lib = None


class ShtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsht error {code}: {msg}")
        self.code = code


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2208_10154_amd.build` "
                               "(hipcc, gfx950); there is no non-HIP fallback")
        L = ctypes.CDLL(LIB_PATH)
        P, I, D, V, S = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.c_size_t
        L.sht_plan_create.argtypes = [ctypes.POINTER(P), I, I, I, I]
        L.sht_plan_create_part.argtypes = [ctypes.POINTER(P), I, I, I, I, I, I]
        L.sht_plan_destroy.argtypes = [P]
        L.sht_plan_set_precision.argtypes = [P, I]
        L.sht_plan_set_stream.argtypes = [P, V]
        L.sht_plan_set_nmaps.argtypes = [P, I]
        L.sht_plan_set_chunk.argtypes = [P, I]
        L.sht_plan_workspace_bytes.argtypes = [P]
        L.sht_plan_workspace_bytes.restype = S
        L.sht_plan_table_bytes.argtypes = [P]
        L.sht_plan_table_bytes.restype = S
        L.sht_plan_ring_rows.argtypes = [P]
        L.sht_plan_ring_rows.restype = ctypes.c_longlong
        L.sht_plan_set_workspace.argtypes = [P, V, S]
        L.sht_alm2map.argtypes = [P, V, V]
        L.sht_alm2map_noalloc.argtypes = [P, V, V]
        L.sht_map2alm.argtypes = [P, V, V]
        L.sht_map2alm_iter.argtypes = [P, V, V, I, D]
        L.sht_alm2map_sel.argtypes = [P, I, V, V]
        L.sht_map2alm_sel.argtypes = [P, I, V, V]
        L.sht_eb_split.argtypes = [P, V, V, V, V]
        L.sht_map2alm_immediate.argtypes = [P, V, V, I, D]
        L.sht_plan_sync.argtypes = [P]
        L.sht_last_error.restype = ctypes.c_char_p
        L.sht_plan_set_profiling.argtypes = [P, I]
        L.sht_plan_get_profile.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong), I]
        for name in EXPORTS:
            if name not in ("sht_plan_workspace_bytes", "sht_plan_table_bytes", "sht_last_error", "sht_plan_ring_rows"):
                getattr(L, name).restype = I
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != SHT_OK:
        raise ShtError(rc, lib().sht_last_error().decode())


COMP_T, COMP_E, COMP_B = 1, 2, 4


def comp_mask(comps: str) -> int:
    """Bit mask of enum sht_comp for a string of component letters ("T", "EB", ...)."""
    bits = {"T": COMP_T, "E": COMP_E, "B": COMP_B}
    if not comps or any(c not in bits for c in comps.upper()):
        raise ValueError(f"components must be letters of 'TEB', got {comps!r}")
    mask = 0
    for c in comps.upper():
        mask |= bits[c]
    return mask


def npix(nside: int) -> int:
    return 12 * nside * nside


def part_orders(lmax: int, part: int, nparts: int) -> list:
    """The orders m a plan of part `part` of `nparts` owns (sht_plan_create_part):
    pairs (q, lmax - q) of the folded order 0, lmax, 1, lmax - 1, ... dealt to the
    parts in turn."""
    ms = set()
    for i in range(lmax + 1):
        if (i >> 1) % nparts == part:
            ms.add(i >> 1 if i % 2 == 0 else lmax - (i >> 1))
    return sorted(ms)


class Plan:
    """One transform plan: nside, lmax, spin (0: T maps, 2: IQU triples) and the
    largest batch of map sets per call."""

    def __init__(self, nside: int, lmax: int, spin: int, nmaps: int, precision: str = "fp64", chunk: int | None = None,
                 part: int | None = None, nparts: int = 1):
        """part/nparts: a plan that owns part `part` of `nparts` of the orders m
        (sht_plan_create_part); by default all of them (sht_plan_create)."""
        self.nside, self.lmax, self.spin, self.capacity = nside, lmax, spin, nmaps
        self.ncomp = 1 if spin == 0 else 3
        self.nmaps = nmaps
        self.part, self.nparts = (0 if part is None else part), nparts
        h = ctypes.c_void_p()
        if part is None and nparts == 1:
            _check(lib().sht_plan_create(ctypes.byref(h), nside, lmax, spin, nmaps))
        else:
            _check(lib().sht_plan_create_part(ctypes.byref(h), nside, lmax, spin, nmaps, self.part, nparts))
        self._h = h
        self.precision = "fp64"
        if precision != "fp64":
            self.set_precision(precision)
        if chunk is not None:
            self.set_chunk(chunk)

    # --- configuration
    def set_precision(self, precision: str) -> None:
        _check(lib().sht_plan_set_precision(self._h, PRECISIONS[precision]))
        self.precision = precision

    def set_chunk(self, maps_per_chunk: int) -> None:
        _check(lib().sht_plan_set_chunk(self._h, int(maps_per_chunk)))

    def set_nmaps(self, n: int) -> None:
        _check(lib().sht_plan_set_nmaps(self._h, int(n)))
        self.nmaps = int(n)

    def set_stream(self, stream) -> None:
        ptr = stream if isinstance(stream, int) else stream.cuda_stream
        _check(lib().sht_plan_set_stream(self._h, ctypes.c_void_p(ptr)))

    def workspace_bytes(self) -> int:
        return int(lib().sht_plan_workspace_bytes(self._h))

    def set_workspace(self, buf=None, nbytes: int | None = None) -> None:
        """Use caller device memory as workspace: a CUDA tensor (kept referenced
        while the plan uses it) or a raw pointer with nbytes; None returns to a
        plan-owned workspace."""
        if buf is None:
            _check(lib().sht_plan_set_workspace(self._h, None, 0))
            self._ws_ref = None
            return
        if isinstance(buf, int):
            ptr, n = buf, int(nbytes)
        else:
            ptr, n = buf.data_ptr(), int(nbytes if nbytes is not None else buf.numel() * buf.element_size())
        _check(lib().sht_plan_set_workspace(self._h, ctypes.c_void_p(ptr), n))
        self._ws_ref = buf

    def table_bytes(self) -> int:
        return int(lib().sht_plan_table_bytes(self._h))

    def ring_rows(self) -> int:
        """(m, ring) rows of ring coefficients the FFT mapping moves per component map."""
        return int(lib().sht_plan_ring_rows(self._h))

    # --- shapes
    def map_shape(self, n: int | None = None):
        return (self.nmaps if n is None else n, self.ncomp, npix(self.nside))

    def alm_shape(self, n: int | None = None):
        return (self.nmaps if n is None else n, self.ncomp, (self.lmax + 1) ** 2)

    def _ptr(self, t, shape, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
        if t.dtype != torch.float64 or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous float64 tensor")
        need = 1
        for s in shape:
            need *= s
        if t.numel() < need:
            raise ValueError(f"{name} holds {t.numel()} values, {need} needed for shape {shape}")
        return ctypes.c_void_p(t.data_ptr())

    def _stream(self, stream):
        import torch
        self.set_stream(stream if stream is not None else torch.cuda.current_stream())

    # --- transforms
    def alm2map(self, alm, maps, stream=None):
        self._stream(stream)
        _check(lib().sht_alm2map(self._h, self._ptr(alm, self.alm_shape(), "alm"), self._ptr(maps, self.map_shape(), "maps")))
        return maps

    def alm2map_noalloc(self, alm, maps, stream=None):
        """sht_alm2map_noalloc: alm2map on the library's static workspace (the call
        allocates no device memory)."""
        self._stream(stream)
        _check(lib().sht_alm2map_noalloc(self._h, self._ptr(alm, self.alm_shape(), "alm"),
                                         self._ptr(maps, self.map_shape(), "maps")))
        return maps

    def map2alm(self, maps, alm, stream=None):
        self._stream(stream)
        _check(lib().sht_map2alm(self._h, self._ptr(maps, self.map_shape(), "maps"), self._ptr(alm, self.alm_shape(), "alm")))
        return alm

    def alm2map_sel(self, comps: str, alm, maps, stream=None):
        """Backward transform of the components named in comps ("T", "E", "B" or a
        combination such as "TE"); see sht_alm2map_sel."""
        self._stream(stream)
        _check(lib().sht_alm2map_sel(self._h, comp_mask(comps), self._ptr(alm, self.alm_shape(), "alm"),
                                     self._ptr(maps, self.map_shape(), "maps")))
        return maps

    def map2alm_sel(self, comps: str, maps, alm, stream=None):
        """Forward transform of the components named in comps; the others are zeroed."""
        self._stream(stream)
        _check(lib().sht_map2alm_sel(self._h, comp_mask(comps), self._ptr(maps, self.map_shape(), "maps"),
                                     self._ptr(alm, self.alm_shape(), "alm")))
        return alm

    def eb_split(self, maps, alm, maps_e, maps_b, stream=None):
        """Pixel-domain E/B separation (spin-2 plans): alm = map2alm(maps),
        maps_e = alm2map(T, E, 0), maps_b = alm2map(0, 0, B)."""
        self._stream(stream)
        shp = self.map_shape()
        _check(lib().sht_eb_split(self._h, self._ptr(maps, shp, "maps"), self._ptr(alm, self.alm_shape(), "alm"),
                                  self._ptr(maps_e, shp, "maps_e"), self._ptr(maps_b, shp, "maps_b")))
        return maps_e, maps_b

    def map2alm_iter(self, maps, alm, niter: int, residuals: bool = False, stream=None):
        self._stream(stream)
        res = (ctypes.c_double * (niter + 1))() if residuals else None
        _check(lib().sht_map2alm_iter(self._h, self._ptr(maps, self.map_shape(), "maps"),
                                      self._ptr(alm, self.alm_shape(), "alm"), int(niter),
                                      ctypes.cast(res, ctypes.POINTER(ctypes.c_double)) if res is not None else None))
        return list(res) if res is not None else None

    def map2alm_immediate(self, maps, alm, niter: int, residuals: bool = False, stream=None):
        """Immediate-mode iteration (Gauss-Seidel sweeps over m); see sht_map2alm_immediate."""
        self._stream(stream)
        res = (ctypes.c_double * (niter + 1))() if residuals else None
        _check(lib().sht_map2alm_immediate(self._h, self._ptr(maps, self.map_shape(), "maps"),
                                           self._ptr(alm, self.alm_shape(), "alm"), int(niter),
                                           ctypes.cast(res, ctypes.POINTER(ctypes.c_double)) if res is not None else None))
        return list(res) if res is not None else None

    def set_profiling(self, enable: bool) -> None:
        _check(lib().sht_plan_set_profiling(self._h, 1 if enable else 0))

    def profile(self, reset: bool = True) -> dict:
        """{stage: (milliseconds, launches)} since the last reset (synchronises)."""
        ms = (ctypes.c_double * len(STAGES))()
        n = (ctypes.c_longlong * len(STAGES))()
        _check(lib().sht_plan_get_profile(self._h, ms, n, 1 if reset else 0))
        return {s: (ms[i], n[i]) for i, s in enumerate(STAGES)}

    def sync(self) -> None:
        _check(lib().sht_plan_sync(self._h))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sht_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
