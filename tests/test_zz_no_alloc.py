"""The allocation-free synthesis entry point (sht_alm2map_noalloc) against the
ordinary one (sht_alm2map) and the oracle, through the C ABI: two calls in a row
on the same plan, the second with a smaller batch, in FP64 (1e-10 against the
oracle) and split BF16 (1e-5), and the size limit of its static workspace."""
import ctypes

import numpy as np
import pytest

import oracle

from .gpu_util import alm_inputs, from_dev, note, rel_rms, to_dev

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "bf16x3": 1e-5}


@pytest.fixture(scope="module")
def sht():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2208_10154_amd import sht as mod
    mod.lib()
    return mod


def _call(sht, p, fn, alm, n):
    import torch
    p.set_nmaps(n)
    p.set_stream(torch.cuda.current_stream())
    maps = torch.full(p.map_shape(n), np.nan, dtype=torch.float64, device="cuda")
    rc = getattr(sht.lib(), fn)(p._h, ctypes.c_void_p(alm.data_ptr()), ctypes.c_void_p(maps.data_ptr()))
    assert rc == sht.SHT_OK, sht.lib().sht_last_error().decode()
    p.sync()
    return from_dev(maps)


@pytest.mark.parametrize("spin,nside,lmax,nmaps,prec", [
    (2, 16, 47, 40, "fp64"),     # 40 map sets: chunks of the static workspace
    (0, 64, 191, 70, "fp64"),
    (2, 16, 47, 40, "bf16x3"),
])
def test_noalloc_matches_alm2map_twice(sht, spin, nside, lmax, nmaps, prec):
    note(f"alm2map_noalloc spin={spin} nside={nside} lmax={lmax} nmaps={nmaps} {prec}")
    a, c = alm_inputs(lmax, nmaps, spin == 2, workload=41)
    alm = to_dev(c)
    p = sht.Plan(nside, lmax, spin, nmaps, precision=prec)
    try:
        for n in (nmaps, 7):  # the second call on a smaller batch
            ref_lib = _call(sht, p, "sht_alm2map", alm, n)
            got = _call(sht, p, "sht_alm2map_noalloc", alm, n)
            assert np.all(np.isfinite(got))
            assert np.all(rel_rms(got, ref_lib) <= TOL[prec])
            ref = (oracle.alm2map_iqu(nside, lmax, a[:n]) if spin == 2
                   else oracle.alm2map(nside, lmax, a[:n, 0])[:, None])
            assert np.all(rel_rms(got, ref) <= TOL[prec])
    finally:
        p.close()


def test_noalloc_refuses_what_does_not_fit(sht):
    """nside 256, lmax 767, spin 0, FP64: one map set needs more workspace than the
    static array holds; the call fails with SHT_ERR_ARG and leaves the output alone."""
    import torch
    note("alm2map_noalloc size limit nside=256 lmax=767")
    p = sht.Plan(256, 767, 0, 1)
    try:
        alm = torch.zeros(p.alm_shape(), dtype=torch.float64, device="cuda")
        maps = torch.full(p.map_shape(), 7.0, dtype=torch.float64, device="cuda")
        rc = sht.lib().sht_alm2map_noalloc(p._h, ctypes.c_void_p(alm.data_ptr()), ctypes.c_void_p(maps.data_ptr()))
        assert rc == sht.SHT_ERR_ARG
        assert "static workspace" in sht.lib().sht_last_error().decode()
        p.sync()
        assert torch.all(maps == 7.0)
    finally:
        p.close()
