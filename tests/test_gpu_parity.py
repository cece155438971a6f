"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars: FP64 <= 1e-10 relative RMS per map and component, FP32 and split-BF16
(BF16x3) <= 1e-5 (the tolerances of the transform's stated parity targets), on
the same seeded inputs.
Sizes span several Legendre tiles (64 l x 32/64 rings), ragged column tiles
(odd map counts), several chunks, Bluestein ring lengths (prime factors > 7)
and odd nside.
"""
import numpy as np
import pytest

import oracle
from paper_2208_10154_amd import synth

from .gpu_util import alm_inputs, from_dev, note, rel_rms, to_dev

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-5}


@pytest.fixture(scope="module")
def sht():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2208_10154_amd import sht as mod
    mod.lib()
    return mod


def run_a2m(sht, nside, lmax, spin, compact, prec="fp64", chunk=None):
    import torch
    n = compact.shape[0]
    p = sht.Plan(nside, lmax, spin, n, precision=prec, chunk=chunk)
    alm = to_dev(compact)
    maps = torch.zeros(p.map_shape(), dtype=torch.float64, device="cuda")
    p.alm2map(alm, maps)
    p.sync()
    out = from_dev(maps)
    p.close()
    return out


def run_m2a(sht, nside, lmax, spin, maps_np, prec="fp64", chunk=None):
    import torch
    n = maps_np.shape[0]
    p = sht.Plan(nside, lmax, spin, n, precision=prec, chunk=chunk)
    maps = to_dev(maps_np)
    alm = torch.full(p.alm_shape(), np.nan, dtype=torch.float64, device="cuda")
    p.map2alm(maps, alm)
    p.sync()
    out = from_dev(alm)
    p.close()
    return out


CASES = [
    # nside, lmax, nmaps, chunk
    (16, 47, 8, None),        # the small FP64 workload (3 nside - 1)
    (13, 38, 5, 2),           # odd nside (Bluestein equator), ragged maps, 3 chunks
    (8, 31, 3, None),         # lmax = 4 nside - 1 (maximum)
    (32, 40, 2, None),        # lmax < 2 nside
    (24, 71, 3, None),        # power-of-two and Bluestein polar rings with lmax >= n (aliased rows)
]


@pytest.mark.parametrize("nside,lmax,nmaps,chunk", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_alm2map_spin0(sht, nside, lmax, nmaps, chunk, prec):
    note(f"alm2map spin0 nside={nside} lmax={lmax} nmaps={nmaps} chunk={chunk} {prec}")
    a, c = alm_inputs(lmax, nmaps, False, workload=1)
    ref = oracle.alm2map(nside, lmax, a[:, 0])
    got = run_a2m(sht, nside, lmax, 0, c, prec, chunk)[:, 0]
    err = rel_rms(got, ref)
    assert np.all(err <= TOL[prec]), err


@pytest.mark.parametrize("nside,lmax,nmaps,chunk", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_map2alm_spin0(sht, nside, lmax, nmaps, chunk, prec):
    note(f"map2alm spin0 nside={nside} lmax={lmax} nmaps={nmaps} chunk={chunk} {prec}")
    a, _ = alm_inputs(lmax, nmaps, False, workload=1)
    maps = oracle.alm2map(nside, lmax, a[:, 0])
    maps = maps + synth.white_noise_like(maps[:, None], 1e-3, workload=1)[:, 0]
    ref = oracle.to_compact(oracle.map2alm(nside, lmax, maps))
    got = run_m2a(sht, nside, lmax, 0, maps[:, None], prec, chunk)[:, 0]
    assert np.all(np.isfinite(got))
    err = rel_rms(got, ref)
    assert np.all(err <= TOL[prec]), err


POL_CASES = [
    (8, 23, 3, None),
    (11, 32, 4, 3),
    (16, 47, 2, None),
    (4, 15, 1, None),
    (24, 71, 2, None),  # aliased rows in the power-of-two and Bluestein ring kernels
    (64, 191, 4, None), # a larger sky: B (a tenth of E's power) held to the bar on its own norm
]


@pytest.mark.parametrize("nside,lmax,nmaps,chunk", POL_CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_alm2map_iqu(sht, nside, lmax, nmaps, chunk, prec):
    note(f"alm2map IQU nside={nside} lmax={lmax} nmaps={nmaps} chunk={chunk} {prec}")
    a, c = alm_inputs(lmax, nmaps, True, workload=2)
    ref = oracle.alm2map_iqu(nside, lmax, a)
    got = run_a2m(sht, nside, lmax, 2, c, prec, chunk)
    err = rel_rms(got, ref)
    assert np.all(err <= TOL[prec]), err


@pytest.mark.parametrize("nside,lmax,nmaps,chunk", POL_CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_map2alm_iqu(sht, nside, lmax, nmaps, chunk, prec):
    note(f"map2alm IQU nside={nside} lmax={lmax} nmaps={nmaps} chunk={chunk} {prec}")
    a, _ = alm_inputs(lmax, nmaps, True, workload=2)
    maps = oracle.alm2map_iqu(nside, lmax, a)
    maps = maps + synth.white_noise_like(maps, 1e-3, workload=2)
    ref = oracle.to_compact(oracle.map2alm_iqu(nside, lmax, maps))
    got = run_m2a(sht, nside, lmax, 2, maps, prec, chunk)
    assert np.all(np.isfinite(got))
    err = rel_rms(got, ref)
    assert np.all(err <= TOL[prec]), err


@pytest.mark.parametrize("pol", [False, True])
def test_map2alm_iter_matches_oracle_jacobi(sht, pol):
    import torch
    nside, lmax, nmaps, niter = 8, 23, 3, 3
    note(f"map2alm_iter pol={pol} nside={nside} lmax={lmax} niter={niter}")
    a, _ = alm_inputs(lmax, nmaps, pol, workload=3)
    maps = oracle.alm2map_iqu(nside, lmax, a) if pol else oracle.alm2map(nside, lmax, a[:, 0])[:, None]
    maps = maps + synth.white_noise_like(maps, 1e-2, workload=3)
    ref_a, ref_res = oracle.map2alm_iter(nside, lmax, maps if pol else maps[:, 0], niter, pol=pol)
    ref = oracle.to_compact(ref_a if pol else ref_a[:, None])
    p = sht.Plan(nside, lmax, 2 if pol else 0, nmaps)
    out = torch.zeros(p.alm_shape(), dtype=torch.float64, device="cuda")
    res = p.map2alm_iter(to_dev(maps), out, niter, residuals=True)
    p.sync()
    got = from_dev(out)
    p.close()
    err = rel_rms(got, ref)
    assert np.all(err <= 1e-10), err
    # oracle residuals are 2-norms over all pixels; the library reports RMS
    rms_ref = np.array(ref_res) / np.sqrt(maps.size)
    np.testing.assert_allclose(res, rms_ref, rtol=1e-9)
    assert all(np.diff(res) < 0)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_map2alm_iter_mixed_precision(sht, prec):
    """Jacobi iteration with the contraction in FP32 / BF16x3 and the residual in
    FP64: the result stays within the mixed-precision bar of the oracle's FP64
    iterates, and the residual still falls every iteration."""
    import torch
    nside, lmax, nmaps, niter = 16, 40, 2, 3
    note(f"map2alm_iter mixed {prec} nside={nside} lmax={lmax} niter={niter}")
    a, _ = alm_inputs(lmax, nmaps, True, workload=5)
    maps = oracle.alm2map_iqu(nside, lmax, a)
    maps = maps + synth.white_noise_like(maps, 1e-2, workload=5)
    ref_a, _ = oracle.map2alm_iter(nside, lmax, maps, niter, pol=True)
    ref = oracle.to_compact(ref_a)
    p = sht.Plan(nside, lmax, 2, nmaps, precision=prec)
    out = torch.zeros(p.alm_shape(), dtype=torch.float64, device="cuda")
    res = p.map2alm_iter(to_dev(maps), out, niter, residuals=True)
    p.sync()
    got = from_dev(out)
    p.close()
    err = rel_rms(got, ref)
    assert np.all(err <= TOL[prec]), err
    assert all(np.diff(res) < 0)


def test_constant_map_analysis_exact(sht):
    """map2alm of the constant map 1: a_00 = sqrt(4 pi); exact zeros (to rounding)
    where the ring sums vanish identically (m not a multiple of 4, odd l at m = 0);
    everything else equals the oracle (quadrature is not exact at even l)."""
    nside, lmax = 16, 47
    note("constant map analysis")
    got = run_m2a(sht, nside, lmax, 0, np.ones((1, 1, 12 * nside * nside)))[0, 0]
    ref = oracle.to_compact(oracle.map2alm(nside, lmax, np.ones((1, 12 * nside * nside))))[0]
    assert abs(got[0] - np.sqrt(4 * np.pi)) < 1e-13
    full = oracle.from_compact(got, lmax)
    for l in range(lmax + 1):
        for m in range(l + 1):
            if m % 4 != 0 or (m == 0 and l % 2 == 1):
                assert abs(full[l, m]) < 1e-13, (l, m, full[l, m])
    assert np.max(np.abs(got - ref)) < 1e-13


def test_batch_position_invariance(sht):
    """A map's result does not depend on which slot of the batch it occupies beyond
    rounding (the ring FFT packs two maps into one complex transform)."""
    nside, lmax = 16, 47
    note("batch invariance")
    a, c = alm_inputs(lmax, 7, True, workload=4)
    full = run_a2m(sht, nside, lmax, 2, c)
    alone = run_a2m(sht, nside, lmax, 2, c[5:6])
    assert np.all(rel_rms(full[5], alone[0]) < 1e-13)


# Small batches: up to 8 map sets run the narrow Legendre tiles (the waves of a
# workgroup split the output blocks of 16 columns) and the ring FFTs skip the
# workgroups that hold only padding map sets; 9 map sets run the 64-column tile.
SMALL = [(48, 143, 1), (48, 143, 8), (33, 98, 9), (16, 63, 3)]
_small_refs = {}


def _small_case(nside, lmax, nmaps, pol):
    """Seeded inputs and the oracle's results for them (shared by the precisions)."""
    key = (nside, lmax, nmaps, pol)
    if key not in _small_refs:
        a, c = alm_inputs(lmax, nmaps, pol, workload=51)
        ref_m = oracle.alm2map_iqu(nside, lmax, a) if pol else oracle.alm2map(nside, lmax, a[:, 0])[:, None]
        maps = synth.white_maps(12 * nside * nside, nmaps, 3 if pol else 1, workload=51)
        ref_a = oracle.to_compact(oracle.map2alm_iqu(nside, lmax, maps) if pol
                                  else oracle.map2alm(nside, lmax, maps[:, 0])[:, None])
        _small_refs[key] = (c, ref_m, maps, ref_a)
    return _small_refs[key]


@pytest.mark.parametrize("nside,lmax,nmaps", SMALL)
@pytest.mark.parametrize("pol", [False, True])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_small_batches_both_directions(sht, nside, lmax, nmaps, prec, pol):
    note(f"small batch pol={pol} nside={nside} lmax={lmax} nmaps={nmaps} {prec}")
    c, ref_m, maps, ref_a = _small_case(nside, lmax, nmaps, pol)
    got_m = run_a2m(sht, nside, lmax, 2 if pol else 0, c, prec)
    assert np.all(rel_rms(got_m, ref_m) <= TOL[prec]), rel_rms(got_m, ref_m)
    got_a = run_m2a(sht, nside, lmax, 2 if pol else 0, maps, prec)
    assert np.all(np.isfinite(got_a))
    assert np.all(rel_rms(got_a, ref_a) <= TOL[prec]), rel_rms(got_a, ref_a)
