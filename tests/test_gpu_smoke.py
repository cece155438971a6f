"""The package's smoke check (one IQU alm2map + map2alm at nside 8 through the C
ABI on cuda:0, compared with the oracle at 1e-10) runs with the GPU suite, so a
failure there shows up beside the parity tests that explain it."""
import pytest

pytestmark = pytest.mark.gpu


def test_smoke_entry_point():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import __graft_entry__
    __graft_entry__.smoke()
