"""Plans that own part of the orders m (sht_plan_create_part), the one-GPU share
of the split by m for resolutions beyond one GPU (Sec. 5):

* small plans: the parts' map2alm outputs, written into one array, give the
  whole plan's a_lm and the oracle's; the parts' alm2map outputs add up to the
  whole synthesis and the oracle's;
* nside 2048, lmax 6143 (the resolution the paper could not hold on one GPU):
  part 0 of 8, one IQU map set, FP64 (1e-10) and BF16x3 (1e-5), sampled a_lm of
  its own m against the oracle and sampled pixels of its partial synthesis
  against the oracle's synthesis of the same m only; the polar rings whose
  Bluestein convolution exceeds the LDS run as four length-n/4 Bluestein DFTs and
  a radix-4 step, and pixels on such rings are among the samples.
"""
import numpy as np
import pytest

import oracle
from paper_2208_10154_amd import synth

from .gpu_util import alm_inputs, from_dev, note, rel_rms, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sht():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2208_10154_amd import sht as mod
    mod.lib()
    return mod


@pytest.mark.parametrize("spin,nside,lmax,nmaps,nparts", [(2, 16, 47, 3, 4), (0, 24, 71, 2, 3)])
def test_parts_assemble_the_whole_transform(sht, spin, nside, lmax, nmaps, nparts):
    import torch
    note(f"part plans spin={spin} nside={nside} lmax={lmax} nparts={nparts}")
    pol = spin == 2
    a, c = alm_inputs(lmax, nmaps, pol, workload=71)
    maps = synth.white_maps(12 * nside * nside, nmaps, 3 if pol else 1, workload=71)
    ref_a = oracle.to_compact(oracle.map2alm_iqu(nside, lmax, maps) if pol
                              else oracle.map2alm(nside, lmax, maps[:, 0])[:, None])
    ref_m = oracle.alm2map_iqu(nside, lmax, a) if pol else oracle.alm2map(nside, lmax, a[:, 0])[:, None]
    whole = sht.Plan(nside, lmax, spin, nmaps)
    w_alm = torch.empty(whole.alm_shape(), dtype=torch.float64, device="cuda")
    whole.map2alm(to_dev(maps), w_alm)
    w_map = torch.empty(whole.map_shape(), dtype=torch.float64, device="cuda")
    whole.alm2map(to_dev(c), w_map)
    whole.sync()
    whole.close()
    alm = torch.full(w_alm.shape, np.nan, dtype=torch.float64, device="cuda")
    msum = torch.zeros(w_map.shape, dtype=torch.float64, device="cuda")
    L1 = lmax + 1
    for k in range(nparts):
        p = sht.Plan(nside, lmax, spin, nmaps, part=k, nparts=nparts)
        before = from_dev(alm)
        p.map2alm(to_dev(maps), alm)
        part_map = torch.full(w_map.shape, np.nan, dtype=torch.float64, device="cuda")
        p.alm2map(to_dev(c), part_map)
        p.sync()
        p.close()
        msum += part_map
        after = from_dev(alm)
        # exactly the entries of this part's m changed
        own = set(sht.part_orders(lmax, k, nparts))
        idx = np.arange(L1 * L1)
        col, row = idx // L1, idx % L1
        m_of = np.where(row >= col, col, L1 - col)
        mine = np.isin(m_of, sorted(own))
        assert np.array_equal(before[..., ~mine], after[..., ~mine], equal_nan=True)
        assert np.all(np.isfinite(after[..., mine]))
    got_a, got_m = from_dev(alm), from_dev(msum)
    assert np.all(np.isfinite(got_a))
    assert np.all(rel_rms(got_a, from_dev(w_alm)) <= 1e-12)
    assert np.all(rel_rms(got_a, ref_a) <= 1e-10)
    assert np.all(rel_rms(got_m, from_dev(w_map)) <= 1e-12)
    assert np.all(rel_rms(got_m, ref_m) <= 1e-10)


def test_part_plans_refuse_the_whole_plan_calls(sht):
    import torch
    note("part plans: unsupported calls")
    p = sht.Plan(8, 23, 2, 1, part=1, nparts=2)
    m = torch.zeros(p.map_shape(), dtype=torch.float64, device="cuda")
    a = torch.zeros(p.alm_shape(), dtype=torch.float64, device="cuda")
    for call in (lambda: p.map2alm_iter(m, a, 1), lambda: p.map2alm_immediate(m, a, 1),
                 lambda: p.eb_split(m, a, torch.zeros_like(m), torch.zeros_like(m)),
                 lambda: p.alm2map_sel("E", a, m), lambda: p.alm2map_noalloc(a, m)):
        with pytest.raises(sht.ShtError) as e:
            call()
        assert e.value.code == sht.SHT_ERR_UNSUPPORTED
    p.close()


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_nside2048_part_sampled(sht, prec):
    import torch
    N, L, nparts = 2048, 6143, 8
    tol = {"fp64": 1e-10, "bf16x3": 1e-5}[prec]
    note(f"part 0 of {nparts}, nside {N} lmax {L}, one IQU map set, {prec}")
    own = sht.part_orders(L, 0, nparts)
    p = sht.Plan(N, L, 2, 1, precision=prec, part=0, nparts=nparts)
    maps_np = synth.white_maps(12 * N * N, 1, 3, workload=72)
    a_out = torch.zeros(p.alm_shape(), dtype=torch.float64, device="cuda")
    p.map2alm(to_dev(maps_np), a_out)
    g = synth.rng(72, 0)
    a_c = np.zeros((3, L + 1, L + 1), dtype=np.complex128)
    samp_m = [0, 2, 3071, 6143, 1, 6142] + [own[k] for k in (7, 100, 300)]
    for mm in samp_m:  # a few columns only, so the synthesis stays cheap to check
        a_c[:, mm:, mm] = g.standard_normal((3, L + 1 - mm)) + 1j * g.standard_normal((3, L + 1 - mm))
    a_c[:, :, 0] = a_c[:, :, 0].real
    a_c[1:, :2, :] = 0
    a_own = a_c.copy()  # what the part synthesises: the other m are ignored
    for mm in samp_m:
        if mm not in own:
            a_own[:, :, mm] = 0
    assert np.any(a_own != a_c)
    m_out = torch.full(p.map_shape(), np.nan, dtype=torch.float64, device="cuda")
    p.alm2map(to_dev(oracle.to_compact(a_c[None])), m_out)
    p.sync()
    p.close()
    # a_lm of own m (including the pole-most and equator-most orders)
    ms = np.array([0, 6143, 8, 6135, own[300], own[300], own[301]])
    ls = np.array([6143, 6143, 5000, 6140, own[300], 6000, 4500])
    assert all(m in own for m in ms)
    L1 = L + 1
    comp = from_dev(a_out[0])
    ref = oracle.analyze_lm(N, L, maps_np[0], ls, ms, pol=True)
    for c in range(3):
        re = comp[c][ms * L1 + ls]
        msafe = np.maximum(ms, 1)
        im = np.where(ms > 0, comp[c][(L1 - msafe) * L1 + (ls - msafe)], 0.0)
        got = re + 1j * im
        assert np.linalg.norm(got - ref[c]) <= tol * np.linalg.norm(ref[c]), (c, got, ref[c])
    # partial synthesis at sampled pixels: the oracle's synthesis of the own m only
    rng = np.random.default_rng(72)
    # fixed pixels on four-step rings (n = 4j beyond the Bluestein LDS plan): ring
    # 1025 (4100 = 4 * 5^2 * 41 pixels) and ring 2039 (8156 pixels, 2039 prime)
    four = [2 * 1025 * 1024 + 7, 2 * 2039 * 2038 + 4000]
    pix = np.concatenate([[0, 3, 12 * N * N - 1, 6 * N * N], four, rng.integers(0, 12 * N * N, 6)])
    got = from_dev(m_out[0][:, pix])
    ref = oracle.synth_pixels(N, L, a_own, pix, pol=True)
    for c in range(3):
        assert np.linalg.norm(got[c] - ref[c]) <= tol * np.linalg.norm(ref[c]), c
