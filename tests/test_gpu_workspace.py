"""Caller-owned workspace (sht_plan_set_workspace).

The transforms give the same results in a caller buffer as in the plan's own
workspace, and match the oracle (FP64 1e-10, FP32 1e-5).  The buffer starts as
all-ones bytes (NaN as doubles), so a read of workspace memory that no kernel
wrote would show.  Refused, each leaving the plan as it was: a misaligned
pointer, a buffer too small, and a later chunk or precision that needs more than
the buffer holds.  The workspace grows with the row pitch of a chunk (64 columns
up to 32 map sets, 128 up to 64) and with the element size of the precision."""
import numpy as np
import pytest

import oracle

from .gpu_util import alm_inputs, from_dev, note, rel_rms, to_dev

pytestmark = pytest.mark.gpu


def test_caller_workspace():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2208_10154_amd import sht
    sht.lib()

    nside, lmax, cap, n = 16, 47, 40, 5
    a, compact = alm_inputs(lmax, n, True, workload=41)
    ref_maps = oracle.alm2map_iqu(nside, lmax, a)
    note(f"caller workspace: nside {nside} lmax {lmax}, capacity {cap}, {n} IQU map sets, chunk 2")
    p = sht.Plan(nside, lmax, 2, cap, chunk=2)
    p.set_nmaps(n)
    alm = to_dev(compact)

    def run():
        maps = torch.zeros(p.map_shape(), dtype=torch.float64, device="cuda")
        back = torch.zeros(p.alm_shape(), dtype=torch.float64, device="cuda")
        p.alm2map(alm, maps)
        p.map2alm(maps, back)
        p.sync()
        return from_dev(maps), from_dev(back)

    def same(res, ref, tol=1e-14):
        return rel_rms(res[0], ref[0]).max() <= tol and rel_rms(res[1], ref[1]).max() <= tol

    own = run()
    assert rel_rms(own[0], ref_maps).max() <= 1e-10
    need = p.workspace_bytes()
    buf = torch.full((need + 512,), 0xFF, dtype=torch.uint8, device="cuda")
    base = (buf.data_ptr() + 255) // 256 * 256

    for ptr, nbytes in ((base + 8, need), (base, need - 1)):
        with pytest.raises(sht.ShtError) as e:
            p.set_workspace(ptr, nbytes)
        assert e.value.code == sht.SHT_ERR_ARG
    assert same(run(), own)

    p.set_workspace(base, need)
    res = run()
    assert same(res, own)
    assert rel_rms(res[0], ref_maps).max() <= 1e-10

    # sized for chunk 2 in FP64: chunk 40 (twice the row pitch) is refused ...
    with pytest.raises(sht.ShtError) as e:
        p.set_chunk(40)
    assert e.value.code == sht.SHT_ERR_ARG
    assert p.workspace_bytes() == need
    # ... but fits in FP32, where FP64 is then refused and FP32 kept
    p.set_precision("fp32")
    p.set_chunk(40)
    assert p.workspace_bytes() == need
    with pytest.raises(sht.ShtError) as e:
        p.set_precision("fp64")
    assert e.value.code == sht.SHT_ERR_ARG
    assert p.workspace_bytes() == need
    res32 = run()
    assert rel_rms(res32[0], ref_maps).max() <= 1e-5
    assert same(res32, own, 1e-5)

    p.set_chunk(2)
    p.set_precision("fp64")
    assert same(run(), own)

    # back to a plan-owned workspace, which can grow
    p.set_workspace(None)
    p.set_chunk(40)
    assert p.workspace_bytes() == 2 * need
    assert same(run(), own)
    p.close()
    del buf
