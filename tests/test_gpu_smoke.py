"""The smoke check of __graft_entry__ (a tiny batched step in both precisions against the
oracle) run as a GPU test, so that the suite sees what the smoke entry point sees."""
import pytest

pytestmark = pytest.mark.gpu


def test_smoke_entry_point():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import __graft_entry__
    __graft_entry__.smoke()
