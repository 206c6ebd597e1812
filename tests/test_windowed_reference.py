"""The factorised full-size reference of tests/windowed.py against the
oracle's plain evolution of the whole chain (CPU)."""
import numpy as np
import pytest

import floquet_inputs as fin
import oracle as O
from tests.windowed import WindowedCircuit


@pytest.mark.parametrize("L,windows,n", [(12, [(1, 3), (6, 8)], 5), (11, [(0, 2), (5, 8)], 4), (9, [(2, 6)], 7)])
def test_windowed_circuit_reference_is_the_oracle_on_a_small_chain(L, windows, n):
    """The factorised reference equals the oracle's full evolution of the
    same gates (every amplitude, every bond), so it can stand in for it on
    chains the oracle cannot hold."""
    wc = WindowedCircuit(L, windows, seed=3 + L)
    sp = fin.random_spinors(L, 4)
    wins, sites = wc.evolve(sp, n)
    ref = O.evolve(O.product_state(sp), L, wc.G, n)
    xs = np.arange(1 << L)
    assert np.max(np.abs(wc.amplitudes(wins, sites, xs) - ref)) < 1e-13
    for b in range(L - 1):
        assert np.max(np.abs(wc.bond_rdm(wins, sites, b) - O.bond_rdm(ref, L, b))) < 1e-13


def test_windowed_circuit_entangles_inside_windows_only():
    """A window's two-site density matrix is mixed after a few periods, a
    bond between factors stays a product of its site matrices."""
    L = 10
    wc = WindowedCircuit(L, [(2, 5)], seed=11)
    sp = fin.random_spinors(L, 12)
    wins, sites = wc.evolve(sp, 3)
    rho_in = wc.bond_rdm(wins, sites, 3)
    assert np.trace(rho_in @ rho_in).real < 0.99
    rho_edge = wc.bond_rdm(wins, sites, 7)
    assert abs(np.trace(rho_edge @ rho_edge).real - 1.0) < 1e-12
