"""The round-end smoke entry point runs and passes on the GPU."""
import pytest

pytestmark = pytest.mark.gpu


def test_smoke_entry_point():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import __graft_entry__ as ge
    ge.smoke()
