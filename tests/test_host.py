"""Host-side logic of the native library, on the CPU: exported symbols, the
FP64 gate builder, the planner and the tile index maps.  Nothing here launches
device work."""
import os
import re

import numpy as np
import pytest
import scipy.linalg as sla

import floquet_inputs as fin
import oracle as O
from tests import plan_tools as pt

pytest.importorskip("torch")
import paper_2111_08044_amd as fl  # noqa: E402
from paper_2111_08044_amd import _native  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _built():
    return os.path.exists(_native.LIB_PATH)


pytestmark = pytest.mark.skipif(not _built(), reason="libfloquet.so not built")


def test_library_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "floquet.h")) as f:
        text = f.read()
    names = set(re.findall(r"^\s*(?:int|int64_t|const char \*)\s*(fl_\w+)\s*\(", text, re.M))
    assert len(names) >= 15
    lib = _native.lib()
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert names == set(_native.SIGNATURES), "binding signatures out of sync with the header"


def test_probe_library_exports_and_validates():
    """libflprobe.so exports what csrc/probe.h declares and rejects
    bad arguments before launching anything."""
    import ctypes
    path = os.path.join(ROOT, "paper_2111_08044_amd", "libflprobe.so")
    if not os.path.exists(path):
        pytest.skip("libflprobe.so not built")
    with open(os.path.join(ROOT, "paper_2111_08044_amd", "csrc", "probe.h")) as f:
        names = set(re.findall(r"^\s*int\s*(flp_\w+)\s*\(", f.read(), re.M))
    assert names == {"flp_fma_loop", "flp_fma_loop_v"}
    lib = ctypes.CDLL(path)
    for n in names:
        assert hasattr(lib, n), n
        f = getattr(lib, n)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        assert f(None, 8, 10, None) == -1
        assert f(ctypes.c_void_p(256), 0, 10, None) == -1
        assert f(ctypes.c_void_p(256), 8, 0, None) == -1
        assert f(ctypes.c_void_p(256), (1 << 20) + 1, 10, None) == -1


def test_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(fl.FloquetError) as e:
        fl.fl_create(12, "c64")
    assert e.value.code == _native.FL_ENODEV


@pytest.mark.parametrize("L", [2, 5, 12])
def test_xyz_bonds_match_oracle(L):
    w = fin.xyz_workload(L)
    got = fl.fl_xyz_bonds(L, w["J"], w["fields"])
    ref = O.xyz_bond_hamiltonians(L, w["J"], w["fields"])
    assert np.max(np.abs(got - ref)) < 1e-15
    gens = fl.fl_xyz_generators(L)
    assert np.max(np.abs(gens - O.xyz_coupling_generators(L))) == 0.0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_host_gates_match_expm_and_are_unitary(seed):
    L = 14
    w = fin.xyz_workload(L, seed=seed)
    h = O.xyz_bond_hamiltonians(L, w["J"], w["fields"])
    for T in (0.25, 1.7):
        G = fl.fl_host_gates(h, T)
        for b in range(L - 1):
            ref = sla.expm(-1j * T / 2 * h[b])
            assert np.max(np.abs(G[b] - ref)) < 1e-14
            assert np.linalg.norm(G[b].conj().T @ G[b] - np.eye(4)) < 2e-15


def test_host_gates_degenerate_and_gue_spectra():
    """Degenerate spectra (SWAP point, zero matrix, diagonal) and the paper's
    random GUE bond terms."""
    X = O.PAULI_X; Y = O.PAULI_Y; Z = O.PAULI_Z
    hs = [2 * np.pi * (np.kron(X, X) + np.kron(Y, Y) + np.kron(Z, Z)), np.zeros((4, 4)),
          np.diag([1.0, 1.0, -2.0, 0.5]).astype(complex)]
    hs += list(2.0 * fin.gue_bond_sample(6))
    for h in hs:
        G = fl.fl_host_gates(np.array([h]), 0.25)[0]
        assert np.max(np.abs(G - sla.expm(-0.125j * h))) < 1e-13


def test_host_ground_states_match_oracle():
    """Lowest eigenvectors of the paper's GUE terms and of the Heisenberg
    bond (singlet at -3), with the same phase convention as the oracle."""
    P = O.PAULIS
    hs = np.array([sum(np.kron(p, p) for p in P)] + list(2.0 * fin.gue_bond_sample(12)))
    g, e = fl.fl_host_ground_states(hs)
    assert abs(e[0] + 3.0) < 1e-13
    for k in range(len(hs)):
        go, eo = O.ground_state(hs[k])
        assert abs(e[k] - eo) < 1e-13
        assert np.max(np.abs(g[k] - go)) < 1e-12
        assert np.max(np.abs(hs[k] @ g[k] - e[k] * g[k])) < 1e-13


def test_thermalization_rate_closed_form():
    """E(t) = E0 on a plateau up to t0, then E0 exp(-Gamma (t - t0)): the
    crossings of E0/e and E0/e^2 are 1/Gamma apart (Sec. IV)."""
    for gamma, t0 in ((0.3, 5.0), (1.3e-4, 200.0)):
        t = np.linspace(0.0, t0 + 4.0 / gamma, 200001)
        E = -2.0 * np.exp(-gamma * np.clip(t - t0, 0.0, None))
        G, t1, t2 = fl.thermalization_rate(t, E)
        assert abs(G / gamma - 1.0) < 1e-6
        assert abs(t1 - (t0 + 1.0 / gamma)) < 1e-4 / gamma
    G, t1, t2 = fl.thermalization_rate([0, 1, 2], [-1.0, -0.5, -0.3])
    assert G is None and t1 is not None and t2 is None
    a, b = fl.fit_exponential_rate([5, 6, 7, 8], np.exp(-2.48 * np.array([5, 6, 7, 8]) + 10.9))
    assert abs(a + 2.48) < 1e-12 and abs(b - 10.9) < 1e-10


def test_host_gate_derivative_matches_expm_frechet():
    L = 6
    w = fin.xyz_workload(L)
    h = O.xyz_bond_hamiltonians(L, w["J"], w["fields"])
    gens = list(O.xyz_coupling_generators(L)[0]) + [h[1], np.kron(O.PAULI_Z, O.PAULI_I)]
    for b in range(L - 1):
        for g in gens:
            dG = fl.fl_host_gate_derivative(h[b], g, 0.25)
            _, ref = sla.expm_frechet(-0.125j * h[b], -0.125j * g)
            assert np.max(np.abs(dG - ref)) < 1e-14
    # degenerate spectrum: sinc limit
    hd = 2 * np.pi * (np.kron(O.PAULI_X, O.PAULI_X) + np.kron(O.PAULI_Y, O.PAULI_Y)
                      + np.kron(O.PAULI_Z, O.PAULI_Z))
    dG = fl.fl_host_gate_derivative(hd, gens[0], 0.25)
    _, ref = sla.expm_frechet(-0.125j * hd, -0.125j * gens[0])
    assert np.max(np.abs(dG - ref)) < 1e-13


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("L", [2, 3, 7, 12, 13, 14, 17, 20])
def test_tile_map_is_a_permutation_with_the_right_bits(dtype, L):
    kmax = 13 if dtype == "c64" else 12
    if L <= kmax:
        hs = [0]
        C, W = L, 0
    else:
        C = 4 if dtype == "c64" else 6    # low bits of the plain sweep's tiles
        W = kmax - C
        hs = list(range(C, L - W + 1))
    for h in hs:
        m = fl.fl_tile_map(L, dtype, h).astype(np.int64)
        assert np.array_equal(np.sort(m), np.arange(1 << L))
        K = C + W
        tiles = m.reshape(-1, 1 << K)
        inside = (1 << C) - 1
        if W:
            inside |= ((1 << W) - 1) << h
        # every tile shares all bits outside the tile set; its elements vary exactly over it
        outside = tiles & ~inside
        assert np.all(outside == outside[:, :1])
        assert np.all(np.bitwise_or.reduce(tiles ^ tiles[:, :1], axis=1) == inside)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("L", [2, 3, 4, 5, 8, 12, 13, 14, 15, 19, 24, 30, 34])
@pytest.mark.parametrize("n", [1, 2, 5, 8, 10, 16, 17, 40])
@pytest.mark.parametrize("dagger", [False, True])
def test_sweep_plan_is_the_brickwork_circuit(dtype, L, n, dagger):
    if dtype == "c128" and L == 34:
        pytest.skip("L = 34 is complex64 only")
    words = fl.fl_plan_query(L, dtype, 0, n, dagger)
    seq = pt.gate_sequence(L, words)
    for b, g, slot in seq:
        assert g == ((L - 1) + b if dagger else b) and slot == -1
    pt.check_trace_equivalent(L, [b for b, _, _ in seq], n, dagger)


@pytest.mark.parametrize("L", [2, 3, 6, 12, 13, 14, 16])
@pytest.mark.parametrize("n", [1, 3, 18])
def test_plan_interpreter_matches_oracle(L, n):
    """Replaying the plan gate by gate on the CPU (a fake device) gives the
    oracle's U_F^n psi0; also for the reverse direction."""
    w = fin.xyz_workload(L)
    hs = O.xyz_bond_hamiltonians(L, w["J"], w["fields"])
    G = O.floquet_gates(hs, w["T"])
    table = np.concatenate([G, np.conj(np.transpose(G, (0, 2, 1)))])
    psi0 = O.product_state(w["spinors"])
    for dagger in (False, True):
        seq = pt.gate_sequence(L, fl.fl_plan_query(L, "c64", 0, n, dagger))
        psi = psi0.copy()
        for b, g, _ in seq:
            psi = O.apply_bond(psi, L, b, table[g])
        ref = O.evolve(psi0, L, G, n, dagger=dagger)
        assert np.linalg.norm(psi - ref) < 1e-12


@pytest.mark.parametrize("L", [2, 3, 9, 12, 13, 20, 24, 30, 34])
@pytest.mark.parametrize("n", [1, 16, 50])
def test_reverse_gradient_plan(L, n):
    """The gradient's reverse pass undoes U_F^n (U_F^dagger order) and every
    op accumulates the bond it undoes."""
    seq = pt.gate_sequence(L, fl.fl_plan_query(L, "c64", 1, n, True))
    for b, g, slot in seq:
        assert g == (L - 1) + b and slot == b
    pt.check_trace_equivalent(L, [b for b, _, _ in seq], n, True)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("L", [2, 3, 12, 13, 14, 21, 30, 34])
def test_energy_cover_visits_every_bond_once(dtype, L):
    if dtype == "c128" and L == 34:
        pytest.skip()
    C, W, R, passes = pt.parse_plan(fl.fl_plan_query(L, dtype, 2, 0, False))
    seen = []
    for k, (h, flags, groups) in enumerate(passes):
        assert flags == (1 if k == 0 else 0)
        for u0, ops in groups:
            assert len(ops) == 1
            i, g, slot = ops[0]
            assert i == 0 and g == -1
            p, p1 = pt.phys_bit(u0, C, h), pt.phys_bit(u0 + 1, C, h)
            assert p1 == p + 1 and slot == L - 2 - p
            seen.append(slot)
    assert sorted(seen) == list(range(L - 1))


@pytest.mark.parametrize("L", [14, 15, 20, 25, 30, 34])
def test_grouped_energy_cover_visits_every_bond_once(L):
    """complex64 cover on 13-bit tiles: every bond exactly once, as op bit i of
    a 5-bit register group inside the tile whose two bits are chain
    neighbours; the first pass also reduces the norm.  At L = 30 the 29 bonds
    take 4 passes (12 bonds in the first, then windows of 6 bonds)."""
    C, W, R, passes = pt.parse_plan(fl.fl_plan_query(L, "c64", 6, 0, False))
    assert (C, W, R) == (6, 7, 5)
    seen = []
    for k, (h, flags, groups) in enumerate(passes):
        assert flags == (1 if k == 0 else 0)
        rows = 0
        for u0, ops in groups:
            assert 0 <= u0 and u0 + R <= C + W and 1 <= len(ops) <= R - 1
            for i, g, slot in ops:
                assert 0 <= i <= R - 2 and g == -1
                p, p1 = pt.phys_bit(u0 + i, C, h), pt.phys_bit(u0 + i + 1, C, h)
                assert p1 == p + 1 and slot == L - 2 - p
                seen.append(slot)
            rows += len(ops)
        assert rows <= C + W - 1
    assert sorted(seen) == list(range(L - 1))
    if L == 30:
        assert len(passes) == 4 and sum(len(o) for _, o in passes[0][2]) == 12


def test_grouped_energy_cover_needs_complex64_and_long_chains():
    with pytest.raises(fl.FloquetError):
        fl.fl_plan_query(13, "c64", 6, 0, False)
    with pytest.raises(fl.FloquetError):
        fl.fl_plan_query(20, "c128", 6, 0, False)


def test_plan_statistics_L30():
    """The fused plan at L = 30 complex64 needs few passes per period: on
    13-bit tiles with 4 low bits (a 9-bit window), 20 passes for a 16-period
    block and 14 for the 10 periods between two energy readouts (31 and 20
    with 6 low bits)."""
    for n, most in ((16, 20), (10, 14)):
        _, _, _, passes = pt.parse_plan(fl.fl_plan_query(30, "c64", 0, n, False))
        assert len(passes) <= most, (n, len(passes))
        gates = sum(len(ops) for _, _, groups in passes for _, ops in groups)
        assert gates == 29 * n


@pytest.mark.parametrize("kind,dtype,geom", [
    (0, "c64", (4, 9, 4)),    # plain sweep: 4 low bits, 4-bit groups (512-thread workgroups)
    (0, "c128", (6, 6, 4)),
    (1, "c64", (4, 8, 4)),    # gradient reverse pass: 12-bit tiles with 4 low bits
    (3, "c64", (4, 9, 4)),    # H0 psi cover of the plain geometry
    (4, "c64", (4, 9, 6)),    # 6-qubit windows
    (5, "c64", (4, 9, 4)),    # 4-qubit windows (forward and reverse pass)
    (6, "c64", (6, 7, 5)),    # energy reduction: 6 low bits, 5-bit groups
])
def test_tile_geometries(kind, dtype, geom):
    """The tile geometry (C low bits, W window bits, R register bits) each
    kind of plan uses at L = 24; the kernels are built for exactly these."""
    C, W, R, _ = pt.parse_plan(fl.fl_plan_query(24, dtype, kind, 2, kind == 1))
    assert (C, W, R) == geom


# ------------------------------------------------------------ dense windows

def _real_form(U):
    """Real 128x128 form with k = 2m + (0 re, 1 im): written out from the
    definition (Re U, -Im U; Im U, Re U) per 2x2 block."""
    A = np.zeros((128, 128))
    A[0::2, 0::2] = U.real
    A[0::2, 1::2] = -U.imag
    A[1::2, 0::2] = U.imag
    A[1::2, 1::2] = U.real
    return A


def _bf16_rne(x):
    """Round float64 values to 8 significant bits, ties to even (numpy)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0
    m, e = np.frexp(x[nz])
    out[nz] = np.ldexp(np.round(np.ldexp(m, 8)), e - 8)   # np.round: half to even
    return out


def _bits_to_f(b):
    return (np.asarray(b, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def test_window_matrix_is_the_product_of_embedded_gates():
    rng = np.random.default_rng(5)
    n = 7
    G = np.array([np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))[0]
                  for _ in range(n)])
    pos = [0, 2, 4, 1, 3, 0, 2]
    U, _ = fl.fl_host_window_matrix(G, pos)
    ref = np.eye(64, dtype=complex)
    for g, p in zip(G, pos):
        # window bit i = site 5 - i of a 6-site chain (MSB first): bits (p, p+1) = bond 4 - p
        ref = O.embed_bond(6, 4 - p, g) @ ref
    assert np.max(np.abs(U - ref)) < 1e-14


@pytest.mark.parametrize("mode", [0, 1])
def test_window_fragments_layout_and_split(mode):
    rng = np.random.default_rng(6)
    G = np.array([np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))[0]
                  for _ in range(5)])
    U, frag = fl.fl_host_window_matrix(G, [0, 1, 2, 3, 4], mode)
    A = _real_form(U)
    w, l = np.meshgrid(np.arange(4), np.arange(64), indexing="ij")
    if mode == 0:
        f = frag.view(np.float32).reshape(4, 64, 64).astype(np.float64)
        kk = np.arange(64)
        ref = A[(32 * w + (l & 31))[..., None], (2 * kk[None, None, :] + (l >> 5)[..., None])]
        assert np.array_equal(f, ref.astype(np.float32).astype(np.float64))
    else:
        # stored: [wave][step][lk][mm][j][c] = part c of U[16 wave + mm][8 step + 4 lk + j]
        assert frag.size == 32768
        hs = _bits_to_f(frag[:16384].view(np.uint16)).reshape(4, 8, 2, 16, 4, 2)
        ls = _bits_to_f(frag[16384:].view(np.uint16)).reshape(4, 8, 2, 16, 4, 2)
        # the lane view the kernel forms: lane l (row 2m' + c', m' = 16 w + (l%32)//2,
        # c' = l % 2, lk = l // 32) takes (Re, -Im) pairs for c' = 0, (Im, Re) for c' = 1
        def lanes(p):
            out = np.zeros((4, 64, 8, 8))
            for ww in range(4):
                for ll in range(64):
                    mm, cr, lk = (ll & 31) >> 1, ll & 1, ll >> 5
                    for stp in range(8):
                        pr = p[ww, stp, lk, mm]              # (4, 2): (Re, Im) per j
                        v = np.stack([pr[:, 0], -pr[:, 1]], 1) if cr == 0 else np.stack([pr[:, 1], pr[:, 0]], 1)
                        out[ww, ll, stp] = v.reshape(8)
            return out
        h, lo = lanes(hs), lanes(ls)
        st, i = np.meshgrid(np.arange(8), np.arange(8), indexing="ij")
        rows = (32 * w + (l & 31))[..., None, None]
        cols = 16 * st[None, None] + 8 * (l >> 5)[..., None, None] + i[None, None]
        a = A[rows, cols]
        assert np.array_equal(h, _bf16_rne(a))
        assert np.array_equal(lo, _bf16_rne(a - h))
        assert np.max(np.abs(a - h - lo)) <= 2.0 ** -17 * np.max(np.abs(a))


@pytest.mark.parametrize("L", [11, 12, 13, 16, 30, 34])
@pytest.mark.parametrize("n", [1, 7, 16, 17])
@pytest.mark.parametrize("dagger", [False, True])
def test_dense_plan_is_the_brickwork_circuit(L, n, dagger):
    words = fl.fl_plan_query(L, "c64", 4, n, dagger)
    C, W, R, passes = pt.parse_plan(words)
    assert R == 6
    seq = pt.gate_sequence(L, words)
    pt.check_trace_equivalent(L, [b for b, _, _ in seq], n, dagger)


def _real_form32(U):
    """Real 32x32 form of a 16x16 complex U, k = 2m + (0 re, 1 im), written out
    from the definition (Re U, -Im U; Im U, Re U) per 2x2 block."""
    A = np.zeros((32, 32))
    A[0::2, 0::2] = U.real
    A[0::2, 1::2] = -U.imag
    A[1::2, 0::2] = U.imag
    A[1::2, 1::2] = U.real
    return A


def test_window4_matrix_and_fragments():
    """4-bit windows: U is the product of the embedded gates (a 4-site chain,
    window bit i = site 3 - i) and lane l, step s holds A[l % 32][2 m + c] for
    m = k' mod 16, c = k' / 16, k' = 2 s + l / 32 (columns component-major)."""
    rng = np.random.default_rng(8)
    G = np.array([np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))[0]
                  for _ in range(5)])
    pos = [0, 2, 1, 0, 2]
    U, frag = fl.fl_host_window_matrix(G, pos, 2)
    ref = np.eye(16, dtype=complex)
    for g, p in zip(G, pos):
        ref = O.embed_bond(4, 2 - p, g) @ ref
    assert U.shape == (16, 16) and np.max(np.abs(U - ref)) < 1e-14
    A = _real_form32(U)
    f = frag.view(np.float32).reshape(64, 16).astype(np.float64)
    l, st = np.meshgrid(np.arange(64), np.arange(16), indexing="ij")
    kc = 2 * st + (l >> 5)
    assert np.array_equal(f, A[l & 31, 2 * (kc & 15) + (kc >> 4)].astype(np.float32).astype(np.float64))
    with pytest.raises(fl.FloquetError):
        fl.fl_host_window_matrix(G, [0, 3], 2)   # gate position outside a 4-bit window


@pytest.mark.parametrize("L", [13, 16, 30, 34])
@pytest.mark.parametrize("n", [1, 7, 16, 17])
@pytest.mark.parametrize("dagger", [False, True])
def test_dense4_plan_is_the_brickwork_circuit(L, n, dagger):
    words = fl.fl_plan_query(L, "c64", 5, n, dagger)
    C, W, R, passes = pt.parse_plan(words)
    assert R == 4 and C + W == 13
    seq = pt.gate_sequence(L, words)
    pt.check_trace_equivalent(L, [b for b, _, _ in seq], n, dagger)


def _window_apply(v, nout, i, G):
    """Apply G (local index 2 bit(i+1) + bit(i)) on bits (i, i+1) of the low
    4-bit window of a (2^nout * 16)-vector."""
    w = v.reshape(1 << nout, 2 ** (2 - i), 2, 2, 1 << i)    # [r, high window bits, bit i+1, bit i, low bits]
    loc = w.reshape(1 << nout, 2 ** (2 - i), 4, 1 << i)       # local index 2 bit(i+1) + bit(i)
    return np.einsum("ab,xhbl->xhal", G, loc).reshape(-1)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_window_overlaps_match_direct_per_op_sums(seed):
    """The reverse pass's overlap terms of a register group from one 16x16
    window overlap Q, against the per-op sums taken directly on the states
    between the gates (what the per-op reverse kernel accumulates)."""
    rng = np.random.default_rng(seed)
    nout, nops = 3, 6
    n = (1 << nout) * 16
    psi = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    lam = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    G = fin.random_unitaries(nops, 4, seed + 10)
    pos = rng.integers(0, 3, nops)
    P, Lm = psi.reshape(1 << nout, 16), lam.reshape(1 << nout, 16)
    Q = P.T @ Lm.conj()                                        # Q[x][y] = sum_r psi_{r,x} conj(lambda_{r,y})
    got = fl.fl_host_window_overlaps(Q, G, pos)
    p, l = psi.copy(), lam.copy()
    for k in range(nops):
        i = int(pos[k])
        loc = lambda v: v.reshape(1 << nout, 2 ** (2 - i), 4, 1 << i)
        M = np.einsum("xhal,xhbl->ab", loc(l).conj(), loc(p))    # M[a][b] = sum conj(lambda_a) psi_b
        ref = [M[a, a].imag for a in range(4)]
        for a in range(4):
            for b in range(a + 1, 4):
                d = M[a, b] - np.conj(M[b, a])
                ref += [d.real, d.imag]
        assert np.max(np.abs(got[k] - np.array(ref))) < 1e-12, k
        p = _window_apply(p, nout, i, G[k])
        l = _window_apply(l, nout, i, G[k])
