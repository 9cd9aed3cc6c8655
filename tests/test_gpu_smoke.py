"""The package entry point's smoke check (one small solve and backward on
cuda:0 against the oracle) runs as part of the GPU suite, so a change that
breaks it shows up with the other GPU tests."""

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def test_smoke_entry_point():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import __graft_entry__
    __graft_entry__.smoke()
