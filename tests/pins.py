"""Pins of the FP64 oracle against results fixed by the paper's definitions and
by mathematics (closed forms, brute force, identities).

Each check returns an error magnitude; the pin tests assert it is tiny and the
planted-mistake tests assert that a plausible mistake planted in the oracle
makes at least one of them large.  `O` is the oracle module (or a patched copy).
"""
from __future__ import annotations

import numpy as np

import floquet_inputs as fin


def dense_vs_gates(O, L, n, seed=7):
    """Gate-by-gate U_F^n psi0 against the dense matrix power built from the
    full layer Hamiltonians, exp(-i T/2 H_second) exp(-i T/2 H_first) (Eq. (3)-(4),
    Sec. III B)."""
    w = fin.xyz_workload(L, seed=seed)
    hs = O.xyz_bond_hamiltonians(L, w["J"], w["fields"])
    G = O.floquet_gates(hs, w["T"])
    psi0 = O.product_state(w["spinors"])
    UF = O.dense_floquet_unitary(L, hs, w["T"])
    ref = np.linalg.matrix_power(UF, n) @ psi0
    got = O.evolve(psi0, L, G, n)
    return np.linalg.norm(got - ref)


def bloch(s):
    """Bloch vector (<X>, <Y>, <Z>) of a unit spinor, written out."""
    a, b = s[0], s[1]
    return np.array([2.0 * (np.conj(a) * b).real, 2.0 * (np.conj(a) * b).imag,
                     abs(a) ** 2 - abs(b) ** 2])


def e0_closed_form(J, fields, spinors):
    """E(0) of a product state: each bond term factorises into Bloch vectors,
    sum_a J^a_b r^a_b r^a_{b+1} + (1/2) f_b.r_b + (1/2) f_{b+1}.r_{b+1}."""
    L = len(spinors)
    r = [bloch(s) for s in spinors]
    E = 0.0
    for b in range(L - 1):
        E += sum(J[b, a] * r[b][a] * r[b + 1][a] for a in range(3))
        E += 0.5 * np.dot(fields[b], r[b]) + 0.5 * np.dot(fields[b + 1], r[b + 1])
    return E


def e0_error(O, L, seed=11):
    w = fin.xyz_workload(L, seed=seed)
    hs = O.xyz_bond_hamiltonians(L, w["J"], w["fields"])
    psi0 = O.product_state(w["spinors"])
    E, N = O.energy(psi0, L, hs)
    return abs(E - e0_closed_form(w["J"], w["fields"], w["spinors"])) + abs(N - 1.0)


def su2_rotation(alpha, nvec):
    """exp(-i alpha n.sigma) = cos(alpha) I - i sin(alpha) n.sigma for a unit n
    (Euler's formula for Pauli vectors)."""
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
    Z = np.array([[1, 0], [0, -1]], dtype=complex)
    ns = nvec[0] * X + nvec[1] * Y + nvec[2] * Z
    return np.cos(alpha) * np.eye(2) - 1j * np.sin(alpha) * ns


def zero_coupling_error(O, L, n, seed=3):
    """J = 0: every gate factorises into single-site rotations, so the state
    stays a product.  Each bond touching site j applies exp(-i (T/2) (1/2) f_j.sigma)
    to it once per period; after n periods site j has turned through the angle
    n * (number of bonds on j) * (T/2) * |f_j| / 2 about f_j.  Energy is conserved."""
    w = fin.xyz_workload(L, seed=seed)
    J0 = np.zeros_like(w["J"])
    hs = O.xyz_bond_hamiltonians(L, J0, w["fields"])
    G = O.floquet_gates(hs, w["T"])
    psi0 = O.product_state(w["spinors"])
    got = O.evolve(psi0, L, G, n)
    tau = w["T"] / 2.0
    sp = []
    for j in range(L):
        nb = (1 if j > 0 else 0) + (1 if j < L - 1 else 0)   # bonds touching j
        f = w["fields"][j]
        fn = np.linalg.norm(f)
        # each touching bond applies exp(-i tau (1/2) f.sigma) once per period
        alpha = n * nb * tau * 0.5 * fn
        sp.append(su2_rotation(alpha, f / fn) @ w["spinors"][j])
    ref = sp[0]
    for s in sp[1:]:
        ref = np.kron(ref, s)
    err_state = np.linalg.norm(got - ref)
    E0, _ = O.energy(psi0, L, hs)
    En, _ = O.energy(got, L, hs)
    return err_state + abs(En - E0)


def ising_error(O, L, n, seed=5):
    """Jx = Jy = 0 and z fields only: U_F is diagonal,
    psi_x(n) = psi_x(0) exp(-i n (T/2) E_x) with
    E_x = sum_b [Jz_b z_b z_{b+1} + (1/2) f_b z_b + (1/2) f_{b+1} z_{b+1}], z = 1 - 2 bit."""
    w = fin.xyz_workload(L, seed=seed)
    J = w["J"].copy()
    J[:, 0] = 0.0
    J[:, 1] = 0.0
    f = w["fields"].copy()
    f[:, 0] = 0.0
    f[:, 1] = 0.0
    hs = O.xyz_bond_hamiltonians(L, J, f)
    G = O.floquet_gates(hs, w["T"])
    psi0 = O.product_state(w["spinors"])
    got = O.evolve(psi0, L, G, n)
    tau = w["T"] / 2.0
    x = np.arange(1 << L)
    z = np.array([1 - 2 * ((x >> (L - 1 - j)) & 1) for j in range(L)], dtype=float)
    Ex = np.zeros(1 << L)
    for b in range(L - 1):
        Ex += J[b, 2] * z[b] * z[b + 1] + 0.5 * f[b, 2] * z[b] + 0.5 * f[b + 1, 2] * z[b + 1]
    ref = psi0 * np.exp(-1j * n * tau * Ex)
    E0, _ = O.energy(psi0, L, hs)
    En, _ = O.energy(got, L, hs)
    return np.linalg.norm(got - ref) + abs(En - E0) + abs(np.vdot(psi0, Ex * psi0).real - E0)


def swap_point_error(O, L, n, seed=9):
    """Jx = Jy = Jz = 2 pi, no fields, T = 1/4: XX + YY + ZZ = 2 SWAP - I, so
    every gate is exp(-i pi/4) SWAP.  The state stays a product of permuted
    spinors: layer 1 swaps sites (b, b+1) for odd b, layer 2 for even b."""
    w = fin.xyz_workload(L, seed=seed)
    J = np.full_like(w["J"], 2.0 * np.pi)
    f = np.zeros_like(w["fields"])
    hs = O.xyz_bond_hamiltonians(L, J, f)
    G = O.floquet_gates(hs, 0.25)
    psi0 = O.product_state(w["spinors"])
    got = O.evolve(psi0, L, G, n)
    order = list(range(L))           # order[j] = which initial spinor sits on site j
    for _ in range(n):
        for parity in (1, 0):
            for b in range(parity, L - 1, 2):
                order[b], order[b + 1] = order[b + 1], order[b]
    ref = np.array([1.0 + 0j])
    for j in range(L):
        ref = np.kron(ref, w["spinors"][order[j]])
    ref = ref * np.exp(-1j * np.pi / 4 * (L - 1) * n)
    return np.linalg.norm(got - ref)


def echo_error(O, L, n, seed=13):
    """(U_F^dagger)^n U_F^n psi0 = psi0 (the echo of Sec. V)."""
    w = fin.xyz_workload(L, seed=seed)
    hs = O.xyz_bond_hamiltonians(L, w["J"], w["fields"])
    G = O.floquet_gates(hs, w["T"])
    psi0 = O.product_state(w["spinors"])
    back = O.echo(psi0, L, G, n)
    return np.linalg.norm(back - psi0)


def energy_dense_error(O, L, seed=17):
    """Bond-sum energy and H0 psi against the dense H0 = sum_b I (x) h_b (x) I."""
    w = fin.xyz_workload(L, seed=seed)
    hs = O.xyz_bond_hamiltonians(L, w["J"], w["fields"])
    psi = fin.random_state(L, seed)
    H = O.dense_h0(L, hs)
    E, N = O.energy(psi, L, hs)
    Ed = np.vdot(psi, H @ psi).real
    hp = O.apply_h0(psi, L, hs)
    rdm_E = sum(np.trace(hs[b] @ O.bond_rdm(psi, L, b)).real for b in range(L - 1))
    return (abs(E - Ed) + np.linalg.norm(hp - H @ psi) + abs(N - np.vdot(psi, psi).real)
            + abs(rdm_E - Ed)) / max(1.0, abs(Ed))


def fd_gradient(O, L, hs_of_theta, theta, T, psi0, n, idx, h):
    """Central difference with one Richardson step (h, h/2) of E_n in theta[idx]
    (idx = len(theta) means T)."""
    def E(th, TT):
        return O.energy_after(L, hs_of_theta(th), TT, psi0, n)

    def D(step):
        if idx == len(theta):
            return (E(theta, T + step) - E(theta, T - step)) / (2 * step)
        tp = theta.copy(); tp[idx] += step
        tm = theta.copy(); tm[idx] -= step
        return (E(tp, T) - E(tm, T)) / (2 * step)

    return (4.0 * D(h / 2) - D(h)) / 3.0


def xyz_theta(J):
    return np.asarray(J, dtype=float).reshape(-1).copy()


def adjoint_fd_error(O, L, n, params, seed=19, h=1e-4):
    """Relative error of the oracle's adjoint gradient against central finite
    differences on a subset of the parameters (couplings and T)."""
    w = fin.xyz_workload(L, seed=seed)
    fields = w["fields"]
    T = w["T"]
    psi0 = O.product_state(w["spinors"])

    def hs_of(th):
        return O.xyz_bond_hamiltonians(L, th.reshape(L - 1, 3), fields)

    theta = xyz_theta(w["J"])
    gens = O.xyz_coupling_generators(L)
    grad, _ = O.adjoint_gradient(L, hs_of(theta), gens, T, psi0, n)
    worst = 0.0
    for idx in params:
        fd = fd_gradient(O, L, hs_of, theta, T, psi0, n, idx, h)
        worst = max(worst, abs(grad[idx] - fd) / max(1e-3, abs(fd)))
    return worst


def full_generators(L, O):
    """Generators of every Hamiltonian parameter written per bond:
    (Jx, Jy, Jz, left field x/y/z, right field x/y/z) -> P = 9, with
    h_b = sum_p theta_{b,p} gens[b, p] exactly."""
    g = np.zeros((L - 1, 9, 4, 4), dtype=complex)
    P = (O.PAULI_X, O.PAULI_Y, O.PAULI_Z)
    for b in range(L - 1):
        for a in range(3):
            g[b, a] = np.kron(P[a], P[a])
            g[b, 3 + a] = 0.5 * np.kron(P[a], O.PAULI_I)
            g[b, 6 + a] = 0.5 * np.kron(O.PAULI_I, P[a])
    return g


def scaling_identity_error(O, L, n, seed=23):
    """Scaling H0 -> c H0 and T -> T/c leaves every gate unchanged and scales
    E by c, so sum_p theta_p dE/dtheta_p - T dE/dT = E over all parameters."""
    w = fin.xyz_workload(L, seed=seed)
    gens = full_generators(L, O)
    theta = np.zeros((L - 1, 9))
    theta[:, 0:3] = w["J"]
    theta[:, 3:6] = w["fields"][:-1]
    theta[:, 6:9] = w["fields"][1:]
    hs = np.einsum("bp,bpij->bij", theta, gens)
    psi0 = O.product_state(w["spinors"])
    grad, E = O.adjoint_gradient(L, hs, gens, w["T"], psi0, n)
    lhs = np.dot(theta.reshape(-1), grad[:-1]) - w["T"] * grad[-1]
    return abs(lhs - E) / max(1.0, abs(E))


def ising_gradient_error(O, L, n, seed=29):
    """Diagonal (Ising) chain: E_n = E_0 for every T, so dE/dT = 0 and
    dE/dJz_b = r^z_b r^z_{b+1} exactly."""
    w = fin.xyz_workload(L, seed=seed)
    J = w["J"].copy(); J[:, :2] = 0.0
    f = w["fields"].copy(); f[:, :2] = 0.0
    hs = O.xyz_bond_hamiltonians(L, J, f)
    psi0 = O.product_state(w["spinors"])
    grad, _ = O.adjoint_gradient(L, hs, O.xyz_coupling_generators(L), w["T"], psi0, n)
    r = [bloch(s) for s in w["spinors"]]
    err = abs(grad[-1])
    for b in range(L - 1):
        err += abs(grad[b * 3 + 2] - r[b][2] * r[b + 1][2])
    return err


def paper_model_error(O, L, omega, seed=31):
    """Largest error of the paper's model in the oracle (Sec. III A-B, IV):
    - U_F^3 v against exp(-i H_o T) exp(-i H_e T) built densely from the GUE
      terms H_k (odd k = even b first in H_o);
    - E(0) of the pair-product ground state of H_o against the closed form
      sum_{odd k} E_gs(H_k) + sum_{even k} tr(h_b (rho_right(m) (x) rho_left(m+1)));
    - the odd-k bond density matrices against the pure pair states."""
    import scipy.linalg as sla
    Hk = np.asarray(fin.gue_bond_sample(L, seed))
    hs, T = O.paper_model(Hk, omega)
    Ho = sum(O.embed_bond(L, b, Hk[b]) for b in range(0, L - 1, 2))
    He = sum(O.embed_bond(L, b, Hk[b]) for b in range(1, L - 1, 2))
    UF = sla.expm(-1j * Ho * T) @ sla.expm(-1j * He * T)
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << L) + 1j * rng.standard_normal(1 << L)
    err = np.max(np.abs(O.evolve(v, L, O.floquet_gates(hs, T), 3) - np.linalg.matrix_power(UF, 3) @ v))
    gs = [O.ground_state(hs[b]) for b in range(0, L - 1, 2)]
    tail = np.array([0.6, 0.8j]) if L % 2 else None
    psi0 = O.pair_product_state([g for g, _ in gs], tail)
    E, N = O.energy(psi0, L, hs)
    rho = [np.outer(g, g.conj()).reshape(2, 2, 2, 2) for g, _ in gs]
    left = [np.einsum("iaja->ij", r) for r in rho]
    right = [np.einsum("aiaj->ij", r) for r in rho]
    if tail is not None:
        left.append(np.outer(tail, tail.conj()))
    Eref = sum(e for _, e in gs)
    for b in range(1, L - 1, 2):
        m = b // 2
        Eref += np.trace(hs[b] @ np.kron(right[m], left[m + 1])).real
    err = max(err, abs(N - 1.0), abs(E - Eref))
    for b in range(0, L - 1, 2):
        g = gs[b // 2][0]
        err = max(err, np.max(np.abs(O.bond_rdm(psi0, L, b) - np.outer(g, g.conj()))))
    return err
