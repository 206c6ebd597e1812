"""Plain FP64 CPU oracle of the Floquet brickwork method.

TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and the cpu_baseline
leg of bench.py may import this module.  The product path (the HIP library and
its Python binding) never imports, links or runs it, and this module shares no
code with it.

Everything here is deliberately slow and literal: NumPy/SciPy in complex128,
one gate at a time, in the order the paper states the circuit.

Conventions (readings of the paper where it leaves a choice open):
  * Sites j = 0..L-1 of an open chain.  The amplitude index is
    x = sum_j bit_j * 2^(L-1-j), i.e. site 0 is the most significant bit,
    matching the bit-string labelling psi_{b1...bL} with b1 leading (Sec. II).
  * Bond b joins sites (b, b+1), b = 0..L-2; this is the paper's 1-indexed
    bond k = b+1 on qubits k, k+1 (Sec. III A).  A bond operator acts on the
    local index 2*bit_b + bit_{b+1}; in Kronecker products the left factor acts
    on site b.
  * Floquet period, Eq. (4): the rightmost product acts first, i.e. the
    gates on the paper's even k (our odd b) are applied first, then the gates
    on odd k (our even b); equivalently U_F = exp(-i H_o T) exp(-i H_e T)
    (Sec. III B).
  * Gate, Eq. (5): a gate evolves its two qubits for half a period under the
    bond Hamiltonian acting during that half, G_b = exp(-i (T/2) h_b).  The
    paper writes this as exp(-i H_k T) with h_b = 2 H_k.  The energy observable
    is H0 = sum_b h_b (the time-averaged Hamiltonian of Eq. (7) up to that
    factor 2).
  * Energy density e = <H0> / (L <psi|psi>); the raw <H0> and <psi|psi> are
    returned alongside.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

# Pauli matrices (sigma, not sigma/2).
PAULI_I = np.eye(2, dtype=np.complex128)
PAULI_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PAULI_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PAULI_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULIS = (PAULI_X, PAULI_Y, PAULI_Z)


# ----------------------------------------------------------------------------
# Model: bond Hamiltonians, gates, initial state (Sec. III A)
# ----------------------------------------------------------------------------

def xyz_bond_hamiltonians(L, J, fields):
    """Bond Hamiltonians of the XYZ-plus-fields chain, shape (L-1, 4, 4).

    h_b = Jx XX + Jy YY + Jz ZZ + (1/2)(f_b . sigma) (x) I + (1/2) I (x) (f_{b+1} . sigma)

    so every interior site receives its full field from its two bonds and the
    two end sites receive half of theirs.
    """
    J = np.asarray(J, dtype=np.float64)
    f = np.asarray(fields, dtype=np.float64)
    hs = np.zeros((L - 1, 4, 4), dtype=np.complex128)
    for b in range(L - 1):
        h = np.zeros((4, 4), dtype=np.complex128)
        for a in range(3):
            h += J[b, a] * np.kron(PAULIS[a], PAULIS[a])
        left = sum(f[b, a] * PAULIS[a] for a in range(3))
        right = sum(f[b + 1, a] * PAULIS[a] for a in range(3))
        h += 0.5 * np.kron(left, PAULI_I) + 0.5 * np.kron(PAULI_I, right)
        hs[b] = h
    return hs


def xyz_coupling_generators(L):
    """d h_b / d J^alpha_b for alpha = x, y, z: shape (L-1, 3, 4, 4)."""
    g = np.zeros((L - 1, 3, 4, 4), dtype=np.complex128)
    for b in range(L - 1):
        for a in range(3):
            g[b, a] = np.kron(PAULIS[a], PAULIS[a])
    return g


def floquet_gates(hs, T):
    """G_b = exp(-i (T/2) h_b) for every bond (Eq. (5))."""
    return np.array([sla.expm(-1j * (T / 2.0) * h) for h in hs])


def product_state(spinors):
    """|psi(0)> = s_0 (x) s_1 (x) ... (x) s_{L-1}, site 0 leftmost (MSB)."""
    psi = np.array([1.0 + 0j])
    for s in spinors:
        psi = np.kron(psi, np.asarray(s, dtype=np.complex128))
    return psi


def ground_state(h):
    """Lowest eigenvector of a Hermitian two-site term (and its eigenvalue),
    unit norm, with its largest component made real and positive."""
    lam, V = np.linalg.eigh(np.asarray(h, dtype=np.complex128))
    g = V[:, 0]
    k = int(np.argmax(np.abs(g)))
    g = g * (np.conj(g[k]) / abs(g[k]))
    return g / np.linalg.norm(g), lam[0]


def pair_product_state(pairs, tail=None):
    """|psi(0)> = (x)_m |d_m> with |d_m> on sites (2m, 2m+1) (Sec. IV, Eq. (9):
    the ground state of the odd-k terms is such a product of two-site ground
    states); for odd L the last site carries the spinor `tail`."""
    psi = np.array([1.0 + 0j])
    for d in pairs:
        psi = np.kron(psi, np.asarray(d, dtype=np.complex128))
    if tail is not None:
        psi = np.kron(psi, np.asarray(tail, dtype=np.complex128))
    return psi


def paper_model(Hk, omega):
    """The paper's circuit (Sec. III A) in this module's conventions: the gate
    exp(-i H_k T) of Eq. (5) is exp(-i (T/2) h_b) with h_b = 2 H_k, and T = 2 pi / omega.
    Returns (h_b list, T).  Its time-averaged Hamiltonian is sum_k H_k = H0 / 2."""
    return [2.0 * np.asarray(H, dtype=np.complex128) for H in Hk], 2.0 * np.pi / omega


def layer_bonds(L, dagger=False):
    """The two layers of one period in application order.

    Forward U_F: odd b (the paper's even k) first, then even b (Eq. (4)).
    U_F^dagger reverses the order: even b first, then odd b.
    """
    odd = [b for b in range(L - 1) if b % 2 == 1]
    even = [b for b in range(L - 1) if b % 2 == 0]
    return (even, odd) if dagger else (odd, even)


# ----------------------------------------------------------------------------
# Gate application (Sec. II, Eq. (2)) and the Floquet period (Eq. (3)-(4))
# ----------------------------------------------------------------------------

def bond_view(psi, L, b):
    """psi as an array (2^b, 4, 2^(L-b-2)): left sites, bond pair, right sites."""
    return psi.reshape(1 << b, 4, 1 << (L - b - 2))


def apply_bond(psi, L, b, G):
    """(G psi) on sites (b, b+1): out[x, i, z] = sum_j G[i, j] psi[x, j, z]."""
    v = bond_view(psi, L, b)
    return np.einsum("ij,xjz->xiz", G, v).reshape(-1)


def floquet_period(psi, L, gates, dagger=False):
    """One application of U_F (or of U_F^dagger) to psi, gate by gate."""
    first, second = layer_bonds(L, dagger)
    for layer in (first, second):
        for b in layer:
            G = gates[b].conj().T if dagger else gates[b]
            psi = apply_bond(psi, L, b, G)
    return psi


def evolve(psi, L, gates, n, dagger=False):
    """U_F^n psi (or (U_F^dagger)^n psi)."""
    for _ in range(n):
        psi = floquet_period(psi, L, gates, dagger)
    return psi


# ----------------------------------------------------------------------------
# Observables (Sec. II Eq. (1); Sec. IV Eq. (10)-(11))
# ----------------------------------------------------------------------------

def inner(phi, psi):
    """<phi|psi> = sum_x conj(phi_x) psi_x (Eq. (1))."""
    return np.vdot(phi, psi)


def bond_rdm(psi, L, b):
    """Two-site reduced density matrix rho_b[i, j] = sum_r psi_{r,i} conj(psi_{r,j})
    (not divided by the norm)."""
    v = bond_view(psi, L, b)
    return np.einsum("xiz,xjz->ij", v, v.conj())


def energy(psi, L, hs):
    """(<psi|H0|psi>, <psi|psi>) with H0 = sum_b h_b, each bond term evaluated
    as sum over the other sites of v^dagger h_b v."""
    E = 0.0
    for b in range(L - 1):
        v = bond_view(psi, L, b)
        hv = np.einsum("ij,xjz->xiz", hs[b], v)
        E += np.vdot(v, hv).real
    return E, np.vdot(psi, psi).real


def energy_density(psi, L, hs):
    """e = <H0> / (L <psi|psi>)."""
    E, N = energy(psi, L, hs)
    return E / (L * N)


def apply_h0(psi, L, hs):
    """H0 psi = sum_b h_b psi (out of place)."""
    out = np.zeros_like(psi)
    for b in range(L - 1):
        out += apply_bond(psi, L, b, hs[b])
    return out


def energy_spread(psi, L, hs):
    """sigma_E = sqrt(<H0^2> - <H0>^2) for a normalised state (Eq. (11)),
    with <H0^2> = ||H0 psi||^2."""
    N = np.vdot(psi, psi).real
    hpsi = apply_h0(psi, L, hs)
    E = np.vdot(psi, hpsi).real / N
    E2 = np.vdot(hpsi, hpsi).real / N
    return np.sqrt(max(E2 - E * E, 0.0)), E, E2


def infidelity(ref, psi):
    """1 - |<ref|psi>|^2 / (<ref|ref> <psi|psi>)."""
    ov = np.vdot(ref, psi)
    return 1.0 - abs(ov) ** 2 / (np.vdot(ref, ref).real * np.vdot(psi, psi).real)


def overlap_error(ref, psi):
    """|1 - <ref|psi>| on the raw vectors (the echo measure of Sec. V)."""
    return abs(1.0 - np.vdot(ref, psi))


def echo(psi0, L, gates, n):
    """Evolve n periods forward with U_F, then n periods back with U_F^dagger
    (Sec. V); returns psi'(0)."""
    psi = evolve(psi0, L, gates, n)
    return evolve(psi, L, gates, n, dagger=True)


def run_energy_series(L, hs, T, spinors, n, every=1):
    """Evolve the product state and record (period, e, <H0>/L, N) every
    `every` periods including period 0."""
    G = floquet_gates(hs, T)
    psi = product_state(spinors)
    rows = []
    for t in range(n + 1):
        if t % every == 0:
            E, N = energy(psi, L, hs)
            rows.append((t, E / (L * N), E / L, N))
        if t < n:
            psi = floquet_period(psi, L, G)
    return psi, rows


# ----------------------------------------------------------------------------
# Dense brute force (the definition |psi(nT)> = U_F^n |psi(0)>, Eq. (3)-(4))
# ----------------------------------------------------------------------------

def embed_bond(L, b, h):
    """The 2^L x 2^L matrix I_{2^b} (x) h (x) I_{2^(L-b-2)}."""
    return np.kron(np.kron(np.eye(1 << b), h), np.eye(1 << (L - b - 2)))


def dense_floquet_unitary(L, hs, T):
    """U_F = exp(-i (T/2) H_second) exp(-i (T/2) H_first) built from the full
    layer Hamiltonians (Sec. III B), for small L."""
    first, second = layer_bonds(L)
    dim = 1 << L
    HA = np.zeros((dim, dim), dtype=np.complex128)
    HB = np.zeros((dim, dim), dtype=np.complex128)
    for b in first:
        HA += embed_bond(L, b, hs[b])
    for b in second:
        HB += embed_bond(L, b, hs[b])
    return sla.expm(-1j * (T / 2.0) * HB) @ sla.expm(-1j * (T / 2.0) * HA)


def dense_h0(L, hs):
    H = np.zeros((1 << L, 1 << L), dtype=np.complex128)
    for b in range(L - 1):
        H += embed_bond(L, b, hs[b])
    return H


# ----------------------------------------------------------------------------
# Reverse-mode gradient of E_n = <psi_n|H0(theta)|psi_n>
# ----------------------------------------------------------------------------

def gate_derivative(h, gen, T):
    """d/dtheta exp(-i (T/2) h(theta)) in the direction dh/dtheta = gen
    (Frechet derivative of the matrix exponential)."""
    tau = T / 2.0
    _, dG = sla.expm_frechet(-1j * tau * h, -1j * tau * gen)
    return dG


def adjoint_gradient(L, hs, gens, T, psi0, n, ckpt_every=None):
    """Gradient of E_n = <psi_n|H0|psi_n>, psi_n = U_F^n psi0, with respect to
    theta_{b,p} (dh_b/dtheta_{b,p} = gens[b, p]) and to the drive period T.

    Method: with the gates g_1..g_M in application order, psi_m = g_m psi_{m-1}
    and lambda_m = g_{m+1}^dagger ... g_M^dagger H0 psi_M,
        dE/dtheta = sum_m 2 Re <lambda_m| (dg_m/dtheta) g_m^dagger |psi_m>
                    + <psi_M| dH0/dtheta |psi_M>.
    Per bond, <lambda|A|psi> = sum_ij A_ij M_ij with
    M_ij = sum_r conj(lambda_{r,i}) psi_{r,j}, accumulated over all periods.
    The states are rebuilt backwards by applying g^dagger; if ckpt_every is
    given, psi is replaced by the forward state stored at every multiple of
    ckpt_every periods.

    Returns (grad[(L-1)*P + 1], E_n); the last entry is dE/dT.
    """
    gens = np.asarray(gens)
    P = gens.shape[1]
    G = floquet_gates(hs, T)
    psi = psi0.copy()
    ckpts = {}
    for t in range(n):
        if ckpt_every and t % ckpt_every == 0:
            ckpts[t] = psi.copy()
        psi = floquet_period(psi, L, G)
    psi_n = psi.copy()
    E, _ = energy(psi_n, L, hs)
    lam = apply_h0(psi_n, L, hs)
    M = np.zeros((L - 1, 4, 4), dtype=np.complex128)
    first, second = layer_bonds(L)
    for t in range(n - 1, -1, -1):
        # undo period t: second layer first, then first layer
        for layer in (second, first):
            for b in layer:
                lv = bond_view(lam, L, b)
                pv = bond_view(psi, L, b)
                M[b] += np.einsum("xiz,xjz->ij", lv.conj(), pv)
                Gd = G[b].conj().T
                psi = apply_bond(psi, L, b, Gd)
                lam = apply_bond(lam, L, b, Gd)
        if ckpt_every and t in ckpts:
            psi = ckpts[t].copy()
    grad = np.zeros((L - 1) * P + 1)
    for b in range(L - 1):
        Gd = G[b].conj().T
        for p in range(P):
            A = gate_derivative(hs[b], gens[b, p], T) @ Gd
            explicit = np.vdot(psi_n, apply_bond(psi_n, L, b, gens[b, p])).real
            grad[b * P + p] = 2.0 * np.sum(A * M[b]).real + explicit
        AT = -0.5j * hs[b]           # (dG/dT) G^dagger = -(i/2) h_b
        grad[-1] += 2.0 * np.sum(AT * M[b]).real
    return grad, E


def energy_after(L, hs, T, psi0, n):
    """E_n = <psi_n|H0|psi_n> by plain forward evolution (for finite differences)."""
    psi = evolve(psi0, L, floquet_gates(hs, T), n)
    return energy(psi, L, hs)[0]


# ----------------------------------------------------------------------------
# Counting helpers (Sec. IV, Fig. 3 caption; Sec. II)
# ----------------------------------------------------------------------------

def gates_per_period(L):
    """Two-qubit gates in one period of the open-chain brickwork: L-1."""
    return L - 1


def gate_count(L, t, T):
    """Gates applied up to time t: g = (L-1) t / T (Fig. 3 caption)."""
    return (L - 1) * t / T


def state_bytes(nqubits, bytes_per_amplitude):
    return (1 << nqubits) * bytes_per_amplitude
