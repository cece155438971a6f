"""Parity of the spin-0 workload at nside 128, lmax 383, 1000 T maps, FP64, in one
batch: four of the maps (first, last and two inside) carry seeded Gaussian a_lm
the oracle also synthesises; the rest hold device-generated coefficients.  The
four are compared in full against the oracle, in both directions."""
import numpy as np
import pytest

import oracle
from paper_2208_10154_amd import synth

from .gpu_util import from_dev, note, rel_rms, to_dev

pytestmark = pytest.mark.gpu

NSIDE, LMAX, NMAPS = 128, 383, 1000
SLOTS = (0, 333, 666, 999)


def test_spin0_nside128_1000_maps():
    import torch
    assert torch.cuda.is_available()
    from paper_2208_10154_amd import sht
    note(f"spin0 nside={NSIDE} lmax={LMAX} nmaps={NMAPS}")
    a = synth.gaussian_alm(LMAX, len(SLOTS), False, workload=2)
    a = a[:, 0] if a.ndim == 4 else a
    ac = oracle.to_compact(a[:, None])
    g = torch.Generator(device="cuda")
    g.manual_seed(2)
    alm = torch.randn((NMAPS, 1, (LMAX + 1) ** 2), generator=g, device="cuda", dtype=torch.float64) * 1e-2
    for i, s in enumerate(SLOTS):
        alm[s] = to_dev(ac[i])
    p = sht.Plan(NSIDE, LMAX, 0, NMAPS)
    maps = torch.full(p.map_shape(), np.nan, dtype=torch.float64, device="cuda")
    p.alm2map(alm, maps)
    out = torch.full(p.alm_shape(), np.nan, dtype=torch.float64, device="cuda")
    p.map2alm(maps, out)
    p.sync()
    got_m = from_dev(maps[list(SLOTS), 0])
    got_a = from_dev(out[list(SLOTS), 0])
    assert bool(torch.isfinite(out).all())
    p.close()
    ref_m = oracle.alm2map(NSIDE, LMAX, a)
    assert np.all(rel_rms(got_m, ref_m) <= 1e-10), rel_rms(got_m, ref_m)
    ref_a = oracle.to_compact(oracle.map2alm(NSIDE, LMAX, got_m)[:, None])[:, 0]
    assert np.all(rel_rms(got_a, ref_a) <= 1e-10), rel_rms(got_a, ref_a)
