"""The smoke entry point (one small forward + adjoint through the autograd function on
colatitudes, checked against the oracle) runs as a GPU test, so that it is exercised with the
rest of the suite."""
import pytest

pytestmark = pytest.mark.gpu


def test_smoke_entry_point():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import __graft_entry__
    __graft_entry__.smoke()
