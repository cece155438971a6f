"""GPU parity on the degenerate sizes: nside 1 and 2 (three and seven rings,
rings of 4 and 8 pixels), lmax 0 for spin 0, the smallest spin-2 band limit
(lmax 2), the largest band limit (4 nside - 1), a single map set, and the
iterative, selective and E/B-separating entry points on the same tiny plans.
FP64: 1e-10 and split BF16: 1e-5 relative RMS per map and component, as in
test_gpu_parity.py."""
import numpy as np
import pytest

import oracle
from paper_2208_10154_amd import synth

from .gpu_util import from_dev, note, rel_rms, to_dev

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "bf16x3": 1e-5}


@pytest.fixture(scope="module")
def sht():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2208_10154_amd import sht as mod
    mod.lib()
    return mod


def white_alm(lmax, n, pol, workload):
    """Unit-variance coefficients at every l (the spectra of synth.gaussian_alm
    start at l = 2, which would leave lmax < 2 empty): m = 0 real, E and B zero
    below l = 2.  Returns (complex [n, ncomp, L+1, L+1], compact)."""
    nc = 3 if pol else 1
    a = np.zeros((n, nc, lmax + 1, lmax + 1), dtype=np.complex128)
    for k in range(n):
        g = synth.rng(workload + 3000, k)
        a[k] = g.standard_normal((nc, lmax + 1, lmax + 1)) + 1j * g.standard_normal((nc, lmax + 1, lmax + 1))
    a *= oracle._tri_mask(lmax)
    a[..., 0] = a[..., 0].real
    if pol:
        a[:, 1:, :2] = 0
    return a, oracle.to_compact(a)


def _plan_run(sht, nside, lmax, spin, n, prec, fn):
    p = sht.Plan(nside, lmax, spin, n, precision=prec)
    try:
        out = fn(p)
        p.sync()
        return out
    finally:
        p.close()


SPIN0 = [(1, 0, 1), (1, 3, 2), (2, 0, 1), (2, 7, 2), (3, 11, 1)]
SPIN2 = [(1, 2, 1), (1, 3, 2), (2, 2, 1), (2, 7, 2)]


@pytest.mark.parametrize("nside,lmax,n", SPIN0)
@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_tiny_spin0_both_directions(sht, nside, lmax, n, prec):
    import torch
    note(f"edge spin0 nside={nside} lmax={lmax} n={n} {prec}")
    a, c = white_alm(lmax, n, False, workload=31)
    ref_m = oracle.alm2map(nside, lmax, a[:, 0])

    def go(p):
        maps = torch.full(p.map_shape(), np.nan, dtype=torch.float64, device="cuda")
        p.alm2map(to_dev(c), maps)
        alm = torch.full(p.alm_shape(), np.nan, dtype=torch.float64, device="cuda")
        p.map2alm(maps, alm)
        return from_dev(maps), from_dev(alm)
    got_m, got_a = _plan_run(sht, nside, lmax, 0, n, prec, go)
    assert np.all(rel_rms(got_m[:, 0], ref_m) <= TOL[prec])
    ref_a = oracle.to_compact(oracle.map2alm(nside, lmax, got_m[:, 0])[:, None])
    assert np.all(np.isfinite(got_a))
    assert np.all(rel_rms(got_a, ref_a) <= TOL[prec])


@pytest.mark.parametrize("nside,lmax,n", SPIN2)
@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_tiny_iqu_both_directions(sht, nside, lmax, n, prec):
    import torch
    note(f"edge IQU nside={nside} lmax={lmax} n={n} {prec}")
    a, c = white_alm(lmax, n, True, workload=32)
    ref_m = oracle.alm2map_iqu(nside, lmax, a)

    def go(p):
        maps = torch.full(p.map_shape(), np.nan, dtype=torch.float64, device="cuda")
        p.alm2map(to_dev(c), maps)
        alm = torch.full(p.alm_shape(), np.nan, dtype=torch.float64, device="cuda")
        p.map2alm(maps, alm)
        return from_dev(maps), from_dev(alm)
    got_m, got_a = _plan_run(sht, nside, lmax, 2, n, prec, go)
    assert np.all(rel_rms(got_m, ref_m) <= TOL[prec])
    ref_a = oracle.to_compact(oracle.map2alm_iqu(nside, lmax, got_m))
    assert np.all(np.isfinite(got_a))
    assert np.all(rel_rms(got_a, ref_a) <= TOL[prec])


def test_tiny_iterations_and_selections(sht):
    import torch
    nside, lmax, n = 2, 7, 2
    note(f"edge iterations / selections nside={nside} lmax={lmax}")
    a, _ = white_alm(lmax, n, True, workload=33)
    maps = oracle.alm2map_iqu(nside, lmax, a) + synth.white_noise_like(oracle.alm2map_iqu(nside, lmax, a), 1e-2,
                                                                      workload=33)
    ref_j, res_j = oracle.map2alm_iter(nside, lmax, maps, 2, pol=True)
    ref_g, res_g = oracle.map2alm_immediate(nside, lmax, maps, 2, pol=True)
    ra, re, rb = oracle.eb_split(nside, lmax, maps)

    def go(p):
        x = to_dev(maps)
        out = {}
        for name in ("iter", "imm"):
            alm = torch.full(p.alm_shape(), np.nan, dtype=torch.float64, device="cuda")
            fn = p.map2alm_iter if name == "iter" else p.map2alm_immediate
            out[name + "_res"] = fn(x, alm, 2, residuals=True)
            out[name] = from_dev(alm)
        alm = torch.full(p.alm_shape(), np.nan, dtype=torch.float64, device="cuda")
        me = torch.full(p.map_shape(), np.nan, dtype=torch.float64, device="cuda")
        mb = torch.full(p.map_shape(), np.nan, dtype=torch.float64, device="cuda")
        p.eb_split(x, alm, me, mb)
        out["eb"] = (from_dev(alm), from_dev(me), from_dev(mb))
        sel = torch.full(p.alm_shape(), np.nan, dtype=torch.float64, device="cuda")
        p.map2alm_sel("B", x, sel)
        out["selB"] = from_dev(sel)
        return out
    out = _plan_run(sht, nside, lmax, 2, n, "fp64", go)
    assert np.all(rel_rms(out["iter"], oracle.to_compact(ref_j)) <= 1e-10)
    assert np.all(rel_rms(out["imm"], oracle.to_compact(ref_g)) <= 1e-10)
    np.testing.assert_allclose(out["iter_res"], res_j / np.sqrt(maps.size), rtol=1e-9)
    np.testing.assert_allclose(out["imm_res"], res_g / np.sqrt(maps.size), rtol=1e-9)
    ga, ge, gb = out["eb"]
    assert np.all(rel_rms(ga, oracle.to_compact(ra)) <= 1e-10)
    assert np.all(rel_rms(ge, re) <= 1e-10)
    assert np.all(gb[:, 0] == 0) and np.all(rel_rms(gb[:, 1:], rb[:, 1:]) <= 1e-10)
    full = oracle.to_compact(ra)
    assert np.all(out["selB"][:, :2] == 0)
    assert np.all(rel_rms(out["selB"][:, 2], full[:, 2]) <= 1e-10)
