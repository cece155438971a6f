"""GPU parity of the immediate-mode iteration (Sec. 4, Algorithm 3) through the C
ABI against the oracle's sequential Gauss-Seidel sweep over m (pinned in
test_oracle_pins.py).  The GPU runs the m of one schedule level together; the
result must still be the sweep's: FP64 <= 1e-10 relative RMS per map and
component, residual RMS to 1e-9; FP32 / BF16x3 within the mixed-precision bar.
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


def _maps(nside, lmax, nmaps, pol, workload, noise=1e-2):
    a, _ = alm_inputs(lmax, nmaps, pol, workload=workload)
    maps = oracle.alm2map_iqu(nside, lmax, a) if pol else oracle.alm2map(nside, lmax, a[:, 0])[:, None]
    return maps + synth.white_noise_like(maps, noise, workload=workload)


def _run(sht, nside, lmax, pol, maps, niter, prec="fp64", chunk=None, immediate=True):
    import torch
    p = sht.Plan(nside, lmax, 2 if pol else 0, maps.shape[0], precision=prec, chunk=chunk)
    out = torch.full(p.alm_shape(), np.nan, dtype=torch.float64, device="cuda")
    fn = p.map2alm_immediate if immediate else p.map2alm_iter
    res = fn(to_dev(maps), out, niter, residuals=True)
    p.sync()
    got = from_dev(out)
    p.close()
    return got, np.array(res)


CASES = [
    # nside, lmax, nmaps, pol, chunk, niter
    (8, 23, 3, True, None, 2),
    (8, 23, 3, True, 2, 1),     # two chunks, ragged last chunk
    (16, 47, 2, False, None, 2),
    (13, 38, 2, True, None, 1),  # odd nside: Bluestein rings, lmax < 3 nside - 1
    (8, 23, 64, True, None, 1),  # 64 map sets: the two-column-tile kernels
]


@pytest.mark.parametrize("nside,lmax,nmaps,pol,chunk,niter", CASES)
def test_immediate_matches_oracle_sweep(sht, nside, lmax, nmaps, pol, chunk, niter):
    note(f"map2alm_immediate nside={nside} lmax={lmax} nmaps={nmaps} pol={pol} chunk={chunk} niter={niter}")
    maps = _maps(nside, lmax, nmaps, pol, workload=21)
    ref_a, ref_res = oracle.map2alm_immediate(nside, lmax, maps if pol else maps[:, 0], niter, pol=pol)
    ref = oracle.to_compact(ref_a if pol else ref_a[:, None])
    got, res = _run(sht, nside, lmax, pol, maps, niter, chunk=chunk)
    err = rel_rms(got, ref)
    assert np.all(err <= 1e-10), err
    np.testing.assert_allclose(res, np.array(ref_res) / np.sqrt(maps.size), rtol=1e-9)


def test_immediate_zero_sweeps_is_map2alm(sht):
    nside, lmax = 8, 23
    note("map2alm_immediate niter=0")
    maps = _maps(nside, lmax, 2, True, workload=22)
    got, res = _run(sht, nside, lmax, True, maps, 0)
    ref = oracle.to_compact(oracle.map2alm_iqu(nside, lmax, maps))
    assert np.all(rel_rms(got, ref) <= 1e-10)
    assert len(res) == 1


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_immediate_mixed_precision(sht, prec):
    nside, lmax, niter = 16, 40, 2
    note(f"map2alm_immediate {prec} nside={nside} lmax={lmax} niter={niter}")
    maps = _maps(nside, lmax, 2, True, workload=23)
    ref_a, _ = oracle.map2alm_immediate(nside, lmax, maps, niter, pol=True)
    got, res = _run(sht, nside, lmax, True, maps, niter, prec=prec)
    assert np.all(rel_rms(got, oracle.to_compact(ref_a)) <= TOL[prec])
    assert np.all(np.diff(res) < 0)


def test_immediate_beats_traditional_on_gpu(sht):
    """Sec. 4's comparison on band-limited maps (lmax = 3 nside - 1): after the
    same number of rounds the immediate residual is well below the traditional one."""
    nside, lmax, niter = 16, 47, 3
    note("immediate vs traditional")
    maps = _maps(nside, lmax, 2, True, workload=24, noise=0.0)
    _, rj = _run(sht, nside, lmax, True, maps, niter, immediate=False)
    _, rg = _run(sht, nside, lmax, True, maps, niter)
    assert rg[0] == pytest.approx(rj[0], rel=1e-12)
    assert rg[-1] < 0.5 * rj[-1], (rg, rj)
