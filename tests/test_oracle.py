"""Pins of the FP64 oracle (CPU only).

The oracle is checked against what the paper's definitions and mathematics fix,
never against itself: dense brute force (Eq. (3)-(4)), closed forms, identities,
finite differences, and the numbers the paper prints.
"""
import json
import os
import types

import numpy as np
import pytest
import scipy.linalg as sla

import floquet_inputs as fin
import oracle as O
from tests import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("L", [2, 3, 4, 5, 6, 7, 8, 9, 10])
def test_gate_by_gate_matches_dense_floquet_unitary(L):
    n = 100 if L <= 8 else 25
    assert pins.dense_vs_gates(O, L, n) < 1e-12


def test_unitarity_over_1000_periods_L12():
    w = fin.xyz_workload(12)
    hs = O.xyz_bond_hamiltonians(12, w["J"], w["fields"])
    G = O.floquet_gates(hs, w["T"])
    for g in G:
        assert np.linalg.norm(g.conj().T @ g - np.eye(4)) < 1e-14
    psi = O.evolve(O.product_state(w["spinors"]), 12, G, 1000)
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-13


@pytest.mark.parametrize("L,n", [(2, 5), (5, 17), (8, 40)])
def test_zero_coupling_closed_form(L, n):
    assert pins.zero_coupling_error(O, L, n) < 1e-12


@pytest.mark.parametrize("L,n", [(3, 9), (8, 33)])
def test_diagonal_ising_closed_form_and_energy_conservation(L, n):
    assert pins.ising_error(O, L, n) < 1e-11


@pytest.mark.parametrize("L,n", [(2, 3), (5, 4), (8, 7), (9, 10)])
def test_swap_point_permutes_spinors(L, n):
    assert pins.swap_point_error(O, L, n) < 1e-12


@pytest.mark.parametrize("L", [2, 5, 10, 12])
def test_initial_energy_closed_form(L):
    assert pins.e0_error(O, L) < 1e-13


def test_echo_returns_initial_state():
    assert pins.echo_error(O, 10, 100) < 1e-12


@pytest.mark.parametrize("L", [3, 6, 8])
def test_bond_sum_energy_matches_dense_h0(L):
    assert pins.energy_dense_error(O, L) < 1e-13


def test_energy_spread_matches_dense():
    L = 7
    w = fin.xyz_workload(L)
    hs = O.xyz_bond_hamiltonians(L, w["J"], w["fields"])
    psi = fin.random_state(L, 3)
    psi = psi / np.linalg.norm(psi)
    H = O.dense_h0(L, hs)
    sig, E, E2 = O.energy_spread(psi, L, hs)
    Ed = np.vdot(psi, H @ psi).real
    E2d = np.vdot(psi, H @ (H @ psi)).real
    assert abs(E - Ed) < 1e-12 and abs(E2 - E2d) < 1e-11
    assert abs(sig - np.sqrt(E2d - Ed ** 2)) < 1e-11


def test_infinite_temperature_energy_is_zero():
    """The bond Hamiltonians are traceless, so the infinite-temperature energy
    tr(H0)/2^L vanishes (Sec. IV, Fig. 3 dashed lines); averaged over all
    computational basis states the oracle's energy must be 0."""
    L = 6
    w = fin.xyz_workload(L)
    hs = O.xyz_bond_hamiltonians(L, w["J"], w["fields"])
    tot = 0.0
    for x in range(1 << L):
        e = np.zeros(1 << L, dtype=complex)
        e[x] = 1.0
        tot += O.energy(e, L, hs)[0]
    assert abs(tot) < 1e-11
    for h in hs:
        assert abs(np.trace(h)) < 1e-15
        assert np.allclose(h, h.conj().T)


def test_adjoint_matches_finite_differences_L6():
    L = 6
    P = 3 * (L - 1)
    assert pins.adjoint_fd_error(O, L, 20, list(range(P + 1))) < 1e-7


def test_adjoint_matches_finite_differences_L10_sampled():
    L = 10
    P = 3 * (L - 1)
    assert pins.adjoint_fd_error(O, L, 20, [0, 4, 11, 13, 26, P]) < 1e-7


def test_adjoint_scaling_identity():
    assert pins.scaling_identity_error(O, 7, 15) < 1e-11


def test_adjoint_diagonal_ising_exact_gradient():
    assert pins.ising_gradient_error(O, 8, 25) < 1e-11


def test_adjoint_with_checkpoints_equals_without():
    L = 8
    w = fin.xyz_workload(L)
    hs = O.xyz_bond_hamiltonians(L, w["J"], w["fields"])
    psi0 = O.product_state(w["spinors"])
    gens = O.xyz_coupling_generators(L)
    g1, E1 = O.adjoint_gradient(L, hs, gens, w["T"], psi0, 30)
    g2, E2 = O.adjoint_gradient(L, hs, gens, w["T"], psi0, 30, ckpt_every=10)
    assert np.max(np.abs(g1 - g2)) < 1e-11 and abs(E1 - E2) < 1e-13


def test_gue_sample_is_traceless_with_frobenius_norm_sqrt2():
    H = fin.gue_bond_sample(12)
    assert H.shape == (11, 4, 4)
    for h in H:
        assert np.allclose(h, h.conj().T, atol=1e-15)
        assert abs(np.trace(h)) < 1e-14
        assert abs(np.linalg.norm(h) - np.sqrt(2.0)) < 1e-14
    # "first L-1 entries of one long list" (Sec. III A)
    assert np.array_equal(fin.gue_bond_sample(5), H[:4])


# ------------------------------------------- the paper's own model (Sec. III A, IV)

def test_ground_state_special_cases():
    # Heisenberg XX + YY + ZZ = 2 SWAP - 1: the singlet (|01> - |10>)/sqrt2 at -3
    P = O.PAULIS
    h = sum(np.kron(p, p) for p in P)
    g, e0 = O.ground_state(h)
    assert abs(e0 + 3.0) < 1e-13
    assert abs(abs(np.vdot(g, np.array([0, 1, -1, 0]) / np.sqrt(2))) - 1.0) < 1e-13
    # a diagonal term: the basis vector of the smallest diagonal entry
    g, e0 = O.ground_state(np.diag([3.0, 1.0, -2.0, 5.0]).astype(complex))
    assert e0 == -2.0 and abs(abs(g[2]) - 1.0) < 1e-15


@pytest.mark.parametrize("L", [6, 7])
def test_pair_product_state_reduces_to_product_state(L):
    s = fin.xyz_workload(L)["spinors"]
    pairs = [np.kron(s[2 * m], s[2 * m + 1]) for m in range(L // 2)]
    tail = s[L - 1] if L % 2 else None
    assert np.max(np.abs(O.pair_product_state(pairs, tail) - O.product_state(s))) < 1e-15


def test_paper_model_floquet_unitary_and_initial_energy():
    """U_F = exp(-i H_o T) exp(-i H_e T) (Sec. III B), the initial energy of the
    ground state of H_o (Eq. (9)) from single-site reduced states, and pure
    odd-k bond states."""
    assert abs(O.paper_model(fin.gue_bond_sample(4), 6.0)[1] - 2 * np.pi / 6.0) < 1e-15
    assert pins.paper_model_error(O, 6, 6.0) < 1e-12
    assert pins.paper_model_error(O, 7, 5.0) < 1e-12


def test_inputs_first_entries_of_one_long_list():
    a = fin.xyz_workload(12)
    b = fin.xyz_workload(30)
    assert np.array_equal(a["fields"], b["fields"][:12])
    assert np.array_equal(a["spinors"], b["spinors"][:12])
    assert np.allclose(np.linalg.norm(b["spinors"], axis=1), 1.0)


def test_paper_printed_numbers():
    """Numbers the paper prints that the counting helpers must reproduce."""
    with open(os.path.join(GOLDEN, "paper_numbers.json")) as f:
        g = json.load(f)
    fig3 = g["fig3_total_gates"]
    T = 2 * np.pi / fig3["omega"]
    got = O.gate_count(fig3["L"], fig3["t"], T)
    assert abs(got - fig3["gates"]) / fig3["gates"] < 0.5 / 42      # printed to 2 digits
    mem = g["sec2_local_branch_bytes"]
    got = O.state_bytes(mem["local_qubits"], mem["bytes_per_amplitude"]) / 1e9
    assert abs(got - mem["gigabytes"]) < 0.05                       # printed to 2 digits
    assert O.gates_per_period(30) == g["gates_per_period_L30"]["gates"]


def test_c1_golden_energy_series():
    """Regression pin: the committed L=12 energy series (written by
    tests/golden/make_golden.py from the oracle) is reproduced."""
    with open(os.path.join(GOLDEN, "c1_energy_L12.json")) as f:
        g = json.load(f)
    L = g["L"]
    w = fin.xyz_workload(L, seed=g["seed"])
    hs = O.xyz_bond_hamiltonians(L, w["J"], w["fields"])
    _, rows = O.run_energy_series(L, hs, w["T"], w["spinors"], g["n"], every=1)
    got = {r[0]: r[1] for r in rows}
    for t, e in g["energy_density"].items():
        assert abs(got[int(t)] - e) < 1e-12


# ---------------------------------------------------------------------------
# Planted mistakes: each plausible bug in the oracle must trip a pin.
# ---------------------------------------------------------------------------

def _mutant(**overrides):
    m = types.SimpleNamespace(**{k: getattr(O, k) for k in dir(O) if not k.startswith("__")})
    for k, v in overrides.items():
        setattr(m, k, v)
    # functions inside the oracle call each other through module globals, so
    # re-bind the composite ones to the mutant's pieces
    def floquet_period(psi, L, gates, dagger=False):
        first, second = m.layer_bonds(L, dagger)
        for layer in (first, second):
            for b in layer:
                G = gates[b].conj().T if dagger else gates[b]
                psi = m.apply_bond(psi, L, b, G)
        return psi

    def evolve(psi, L, gates, n, dagger=False):
        for _ in range(n):
            psi = m.floquet_period(psi, L, gates, dagger)
        return psi

    if "floquet_period" not in overrides:
        m.floquet_period = floquet_period
    m.evolve = evolve
    m.echo = lambda psi0, L, gates, n: evolve(evolve(psi0, L, gates, n), L, gates, n, True)
    return m


def _all_pins(m):
    return max(pins.dense_vs_gates(m, 5, 7), pins.swap_point_error(m, 5, 3),
               pins.zero_coupling_error(m, 5, 5), pins.e0_error(m, 5),
               pins.ising_error(m, 4, 5))


def test_planted_transposed_gate_is_caught():
    def apply_bond(psi, L, b, G):
        v = O.bond_view(psi, L, b)
        return np.einsum("ij,xjz->xiz", G.T, v).reshape(-1)
    assert _all_pins(_mutant(apply_bond=apply_bond)) > 1e-3


def test_planted_swapped_layer_order_is_caught():
    def layer_bonds(L, dagger=False):
        a, b = O.layer_bonds(L, dagger)
        return b, a
    assert pins.dense_vs_gates(_mutant(layer_bonds=layer_bonds), 5, 7) > 1e-3


def test_planted_reversed_bit_order_is_caught():
    def product_state(spinors):
        return O.product_state(spinors[::-1])
    m = _mutant(product_state=product_state)
    assert max(pins.swap_point_error(m, 5, 3), pins.e0_error(m, 5)) > 1e-3


def test_planted_dropped_field_is_caught():
    def xyz_bond_hamiltonians(L, J, fields):
        f = np.array(fields, dtype=float)
        f[-1] = 0.0
        return O.xyz_bond_hamiltonians(L, J, f)
    assert pins.e0_error(_mutant(xyz_bond_hamiltonians=xyz_bond_hamiltonians), 5) > 1e-3


def test_planted_sign_of_exponent_is_caught():
    import scipy.linalg as sla

    def floquet_gates(hs, T):
        return np.array([sla.expm(+1j * (T / 2.0) * h) for h in hs])
    assert pins.zero_coupling_error(_mutant(floquet_gates=floquet_gates), 5, 5) > 1e-3


def test_planted_full_period_gate_time_is_caught():
    import scipy.linalg as sla

    def floquet_gates(hs, T):
        return np.array([sla.expm(-1j * T * h) for h in hs])
    m = _mutant(floquet_gates=floquet_gates)
    assert max(pins.zero_coupling_error(m, 5, 5), pins.ising_error(m, 4, 5)) > 1e-3


def test_planted_missing_conjugate_in_adjoint_is_caught():
    src_M = O.adjoint_gradient

    def adjoint_gradient(L, hs, gens, T, psi0, n, ckpt_every=None):
        # the same method with conj(lambda) replaced by lambda
        G = O.floquet_gates(hs, T)
        psi = O.evolve(psi0, L, G, n)
        psi_n = psi.copy()
        E, _ = O.energy(psi_n, L, hs)
        lam = O.apply_h0(psi_n, L, hs)
        M = np.zeros((L - 1, 4, 4), dtype=complex)
        first, second = O.layer_bonds(L)
        for t in range(n):
            for layer in (second, first):
                for b in layer:
                    M[b] += np.einsum("xiz,xjz->ij", O.bond_view(lam, L, b), O.bond_view(psi, L, b))
                    Gd = G[b].conj().T
                    psi = O.apply_bond(psi, L, b, Gd)
                    lam = O.apply_bond(lam, L, b, Gd)
        P = gens.shape[1]
        grad = np.zeros((L - 1) * P + 1)
        for b in range(L - 1):
            for p in range(P):
                A = O.gate_derivative(hs[b], gens[b, p], T) @ G[b].conj().T
                grad[b * P + p] = 2 * np.sum(A * M[b]).real + np.vdot(
                    psi_n, O.apply_bond(psi_n, L, b, gens[b, p])).real
            grad[-1] += 2 * np.sum(-0.5j * hs[b] * M[b]).real
        return grad, E
    assert src_M is O.adjoint_gradient
    assert pins.adjoint_fd_error(_mutant(adjoint_gradient=adjoint_gradient), 5, 6, [0, 5, 12]) > 1e-3


def test_infidelity_and_overlap_error_special_cases():
    """Infidelity vanishes for the same ray (any phase and scale), is 1 for
    orthogonal states and 1/2 for states at 45 degrees; the echo overlap error
    |1 - <a|b>| is 0 only for identical normalised vectors."""
    a = fin.random_state(6, 1)
    a = a / np.linalg.norm(a)
    assert abs(O.infidelity(a, 2.5 * np.exp(0.7j) * a)) < 1e-15
    b = np.zeros(4, complex); b[0] = 1
    c = np.zeros(4, complex); c[1] = 1j
    assert abs(O.infidelity(b, c) - 1.0) < 1e-15
    assert abs(O.infidelity(b, (b + c) / np.sqrt(2)) - 0.5) < 1e-15
    assert O.overlap_error(a, a) < 1e-15
    assert abs(O.overlap_error(a, np.exp(0.1j) * a) - abs(1 - np.exp(0.1j))) < 1e-15


def test_planted_swapped_pair_index_is_caught():
    def pair_product_state(pairs, tail=None):
        return O.pair_product_state([np.asarray(d).reshape(2, 2).T.reshape(4) for d in pairs], tail)
    assert pins.paper_model_error(_mutant(pair_product_state=pair_product_state), 6, 6.0) > 1e-3


def test_planted_full_strength_paper_gate_is_caught():
    def paper_model(Hk, omega):
        return [np.asarray(H, dtype=np.complex128) for H in Hk], 2.0 * np.pi / omega
    assert pins.paper_model_error(_mutant(paper_model=paper_model), 6, 6.0) > 1e-3
