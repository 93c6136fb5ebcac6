"""The smoke entry point (one small SGP solve checked against the oracle) runs and passes on the GPU."""
import pytest

pytestmark = pytest.mark.gpu


def test_smoke_entry_point():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import __graft_entry__ as ge
    ge.smoke()
