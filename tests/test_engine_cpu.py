"""Host-side checks of the Python wrappers that need neither a GPU nor the
built library: the autograd function rejects a checkpoint interval that does
not divide the depth before it evolves anything."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2111_08044_amd.engine import FloquetEnergy  # noqa: E402


class _NoEngine:
    """Stands in for a FloquetEngine: any use of it fails the test."""
    L = 6

    def __getattr__(self, name):
        raise AssertionError(f"the engine was used ({name}) before the depth was checked")


@pytest.mark.parametrize("n,K", [(10, 3), (7, 2), (3, 5), (-1, 0), (4, -2)])
def test_floquet_energy_rejects_bad_checkpoint_interval(n, K):
    J = torch.zeros(5, 3, dtype=torch.float64, requires_grad=True)
    T = torch.tensor(0.25, dtype=torch.float64, requires_grad=True)
    with pytest.raises(ValueError):
        FloquetEnergy.apply(J, T, _NoEngine(), np.zeros((6, 3)), np.ones((6, 2)), n, K)


@pytest.mark.parametrize("n,K", [(0, 0), (0, 5), (10, 0), (10, 5), (200, 50), (6, 6)])
def test_floquet_energy_accepts_dividing_interval(n, K):
    assert FloquetEnergy.check_depth(n, K) == (n, K)
