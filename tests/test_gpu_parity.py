"""GPU parity of the HIP path against the FP64 oracle (MI355X only).

Every call goes through the C ABI.  Small chains are compared element by
element; full-size chains (L = 30, the benchmark's plan and launch shapes) are
compared on outputs the oracle can compute exactly: bond density matrices of
a light-cone subchain, closed forms and the echo.
"""
import os
import sys

import numpy as np
import pytest

import floquet_inputs as fin
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2111_08044_amd as fl  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _gpu_state(ctx, vec=None):
    psi = fl.new_state(ctx)
    if vec is not None:
        psi.copy_(torch.from_numpy(np.asarray(vec, dtype=np.complex128)).to(psi.dtype))
    return psi


def _model(L, seed=fin.DEFAULT_SEED, T=0.25):
    w = fin.xyz_workload(L, seed=seed, T=T)
    hs = O.xyz_bond_hamiltonians(L, w["J"], w["fields"])
    return w, hs


# ----------------------------------------------------------------- C1 parity

def test_c1_fp64_state_and_energy_over_1000_periods():
    """L = 12 complex128, identical FP64 gates on both sides: the state after
    1000 periods within 1e-12 in L2 and e(t) within 1e-12 every period."""
    L, n = 12, 1000
    say("case: C1 fp64 L=12 n=1000")
    w, hs = _model(L)
    G = O.floquet_gates(hs, w["T"])
    ctx = fl.fl_create(L, "c128")
    fl.fl_set_gates(ctx, G, hs, w["T"])
    psi = _gpu_state(ctx)
    fl.fl_init_state(ctx, psi, w["spinors"])
    ref = O.product_state(w["spinors"])
    assert np.linalg.norm(psi.cpu().numpy() - ref) < 1e-15
    worst_e = 0.0
    for t in range(1, n + 1):
        fl.fl_apply_period(ctx, psi, 1)
        ref = O.floquet_period(ref, L, G)
        E, N = fl.fl_expect_energy(ctx, psi)
        Er, Nr = O.energy(ref, L, hs)
        worst_e = max(worst_e, abs(E / (L * N) - Er / (L * Nr)))
    err = np.linalg.norm(psi.cpu().numpy() - ref)
    say(f"C1 fp64: state L2 {err:.3e}, worst e {worst_e:.3e}, |N-1| {abs(N - 1):.3e}")
    assert err < 1e-12
    assert worst_e < 1e-12
    assert abs(N - 1.0) < 1e-13


def test_c1_fp32_energy_density_after_1000_periods():
    """L = 12 complex64 with the library's own gates (fl_set_bonds): energy
    density within 1e-5 of the oracle every 10 periods up to 1000."""
    L, n = 12, 1000
    say("case: C1 fp32 L=12 n=1000")
    w, hs = _model(L)
    ctx = fl.fl_create(L, "c64")
    fl.fl_set_bonds(ctx, fl.fl_xyz_bonds(L, w["J"], w["fields"]), w["T"])
    psi = _gpu_state(ctx)
    fl.fl_init_state(ctx, psi, w["spinors"])
    _, rows = O.run_energy_series(L, hs, w["T"], w["spinors"], n, every=10)
    worst = 0.0
    for t, e_ref, _, _ in rows:
        if t > 0:
            fl.fl_apply_period(ctx, psi, 10)
        E, N = fl.fl_expect_energy(ctx, psi)
        worst = max(worst, abs(E / (L * N) - e_ref))
    say(f"C1 fp32: worst |e - e_ref| {worst:.3e}, final |N-1| {abs(N - 1):.3e}")
    assert worst < 1e-5


# ----------------------------------------------------- small and ragged chains

@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("L", [2, 3, 4, 5, 9, 13, 14, 15, 17])
def test_small_chains_element_by_element(dtype, L):
    """Single-tile, multi-tile and ragged plans (n = 1, 7, 17 so that blocks of
    16 periods and remainders both run) against the oracle."""
    say(f"case: small L={L} {dtype}")
    w, hs = _model(L, seed=100 + L)
    G = O.floquet_gates(hs, w["T"])
    ctx = fl.fl_create(L, dtype)
    fl.fl_set_gates(ctx, G, hs, w["T"])
    psi = _gpu_state(ctx)
    fl.fl_init_state(ctx, psi, w["spinors"])
    ref = O.product_state(w["spinors"])
    tol = 1e-12 if dtype == "c128" else 3e-6
    for n in (1, 7, 17):
        fl.fl_apply_period(ctx, psi, n)
        ref = O.evolve(ref, L, G, n)
        got = psi.cpu().numpy().astype(np.complex128)
        assert np.max(np.abs(got - ref)) < tol, (n, np.max(np.abs(got - ref)))
    # and back with U_F^dagger
    fl.fl_apply_period(ctx, psi, 25, dagger=True)
    ref = O.product_state(w["spinors"])
    got = psi.cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(got - ref)) < 10 * tol


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("L", [2, 6, 13, 14, 16, 21])
def test_rdm_energy_and_spread_match_oracle(dtype, L):
    """Bond density matrices, energy, norm and spread against the oracle on a
    random (non-product) state.  complex64 from L = 14 up runs the 13-bit-tile
    register-group readout (L = 14: two tiles), below it the 12-bit forms."""
    say(f"case: rdm L={L} {dtype}")
    w, hs = _model(L, seed=7)
    rng = np.random.default_rng(L)
    v = rng.standard_normal(1 << L) + 1j * rng.standard_normal(1 << L)
    ctx = fl.fl_create(L, dtype)
    fl.fl_set_bonds(ctx, hs, w["T"])
    psi = _gpu_state(ctx, v)
    vv = psi.cpu().numpy().astype(np.complex128)   # what the GPU actually holds
    E, N, rho = fl.fl_expect_energy(ctx, psi, rdm=True)
    Er, Nr = O.energy(vv, L, hs)
    # Both precisions sum in FP64; complex64 amplitudes are widened first, so
    # every product is exact and only FP64 additions round.  The sums run as
    # per-lane chains of at most 64 terms and trees above them (wave, tiles,
    # workgroups), so the error is below ~100 * 2^-53 times the sum of the
    # terms' magnitudes, which is at most N for every entry: 1e-12 N holds.
    rtol = 1e-13 if dtype == "c128" else 1e-12
    assert abs(N - Nr) < rtol * Nr
    assert abs(E - Er) < rtol * Nr * L
    for b in range(L - 1):
        assert np.max(np.abs(rho[b] - O.bond_rdm(vv, L, b))) < rtol * Nr
    ws = _gpu_state(ctx)
    E1, E2, N2 = fl.fl_energy_spread(ctx, psi, ws)
    hv = O.apply_h0(vv, L, hs)
    assert abs(E1 - np.vdot(vv, hv).real) < 1e-5 * Nr * L
    assert abs(E2 - np.vdot(hv, hv).real) < 1e-5 * np.vdot(hv, hv).real
    if dtype == "c128":
        assert np.max(np.abs(ws.cpu().numpy() - hv)) < 1e-12 * np.max(np.abs(hv))


# ------------------------------------------- the paper's own model (Sec. III A, IV)

@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("L", [12, 13])
def test_pair_init_matches_oracle(dtype, L):
    say(f"case: pair init L={L} {dtype}")
    hs = O.paper_model(fin.gue_bond_sample(L), 6.0)[0]
    pairs = [O.ground_state(hs[b])[0] for b in range(0, L - 1, 2)]
    tail = np.array([0.6, 0.8j]) if L % 2 else None
    ctx = fl.fl_create(L, dtype)
    psi = _gpu_state(ctx)
    fl.fl_init_pairs(ctx, psi, np.array(pairs), tail)
    ref = O.pair_product_state(pairs, tail)
    tol = 1e-15 if dtype == "c128" else 1e-7
    assert np.max(np.abs(psi.cpu().numpy() - ref)) < tol


@pytest.mark.parametrize("dtype,n", [("c128", 40), ("c64", 300)])
def test_paper_model_circuit_matches_oracle(dtype, n):
    """The paper's GUE circuit at omega = 6 from the ground state of H_o:
    state, E and sigma_E against the oracle (FP64: state L2 1e-12; FP32:
    energy density 1e-5)."""
    L, omega = 12, 6.0
    say(f"case: paper model L={L} {dtype} n={n}")
    Hk = fin.gue_bond_sample(L)
    hs, T = O.paper_model(Hk, omega)
    eng = fl.FloquetEngine(L, dtype)
    eng.set_paper_model(Hk, omega)
    psi = eng.new_state()
    eng.init_ground_pairs(psi)
    ref = O.pair_product_state([O.ground_state(hs[b])[0] for b in range(0, L - 1, 2)])
    ref = O.evolve(ref, L, O.floquet_gates(hs, T), n)
    eng.step(psi, n)
    got = psi.cpu().numpy().astype(np.complex128)
    if dtype == "c128":
        assert np.linalg.norm(got - ref) < 1e-12
    e_ref = O.energy_density(ref, L, hs)
    assert abs(eng.energy_density(psi) - e_ref) < (1e-12 if dtype == "c128" else 1e-5)
    ws = eng.new_state()
    sig, e1, e2 = eng.energy_spread(psi, ws)
    sig_ref = O.energy_spread(ref, L, hs)[0]
    assert abs(sig - sig_ref) < (1e-10 if dtype == "c128" else 1e-4) * max(1.0, sig_ref)


def test_overlap_mixed_precision():
    L = 15
    rng = np.random.default_rng(3)
    a = rng.standard_normal(1 << L) + 1j * rng.standard_normal(1 << L)
    b = rng.standard_normal(1 << L) + 1j * rng.standard_normal(1 << L)
    ctx = fl.fl_create(L, "c64")
    ta = torch.from_numpy(a).cuda()                      # complex128
    tb = torch.from_numpy(b).to(torch.complex64).cuda()  # complex64
    bb = tb.cpu().numpy().astype(np.complex128)
    ov, na, nb = fl.fl_overlap(ctx, ta, tb)
    assert abs(ov - np.vdot(a, bb)) < 1e-12 * np.sqrt(na * nb)
    assert abs(na - np.vdot(a, a).real) < 1e-12 * na
    assert abs(nb - np.vdot(bb, bb).real) < 1e-12 * nb


# ------------------------------------------- full size (L = 30, bench plan)

def _lightcone_rdm(L, hs, G, spinors, n, b):
    """rho_b after n periods from the oracle on the subchain that holds the
    backward light cone of bond b (2n sites each side; even start keeps the
    layer parity of every bond)."""
    lo = max(0, b - 2 * n - 1)
    lo -= lo % 2
    hi = min(L - 1, b + 1 + 2 * n + 1)
    Ls = hi - lo + 1
    psi = O.product_state(spinors[lo:hi + 1])
    psi = O.evolve(psi, Ls, G[lo:hi], n)
    return O.bond_rdm(psi, Ls, b - lo)


@pytest.mark.parametrize("n", [3])
def test_L30_lightcone_rdms_fp32(n):
    """L = 30 complex64 through the benchmark's plan and kernels: bond density
    matrices after n periods against the oracle on light-cone subchains."""
    L = 30
    say(f"case: L=30 light cone n={n}")
    w, hs = _model(L)
    G = O.floquet_gates(hs, w["T"])
    ctx = fl.fl_create(L, "c64")
    fl.fl_set_bonds(ctx, fl.fl_xyz_bonds(L, w["J"], w["fields"]), w["T"])
    psi = fl.new_state(ctx)
    fl.fl_init_state(ctx, psi, w["spinors"])
    fl.fl_apply_period(ctx, psi, n)
    E, N, rho = fl.fl_expect_energy(ctx, psi, rdm=True)
    worst = 0.0
    for b in (0, 1, 6, 11, 12, 13, 14, 19, 20, 27, 28):
        ref = _lightcone_rdm(L, hs, G, w["spinors"], n, b)
        worst = max(worst, np.max(np.abs(rho[b] - ref)))
    say(f"L=30 light-cone rdm worst {worst:.3e}, |N-1| {abs(N - 1):.3e}")
    assert worst < 2e-6
    assert abs(N - 1) < 1e-5
    del psi
    torch.cuda.empty_cache()


def test_L34_in_place_lightcone_rdms_fp32():
    """The largest chain (L = 34, a 128 GiB complex64 state in place, the
    long-run size): bond density matrices after 2 periods of the 16-period
    plan's prefix, against the oracle on light-cone subchains, every bond."""
    L, n = 34, 2
    free, total = torch.cuda.mem_get_info()
    if free < (1 << L) * 8 + (8 << 30):
        pytest.skip(f"needs 136 GiB of free device memory, {free / 2**30:.0f} GiB free")
    say(f"case: L=34 light cone n={n}")
    w, hs = _model(L)
    G = O.floquet_gates(hs, w["T"])
    ctx = fl.fl_create(L, "c64")
    fl.fl_set_bonds(ctx, fl.fl_xyz_bonds(L, w["J"], w["fields"]), w["T"])
    psi = fl.new_state(ctx)
    try:
        fl.fl_init_state(ctx, psi, w["spinors"])
        fl.fl_apply_period(ctx, psi, n)
        E, N, rho = fl.fl_expect_energy(ctx, psi, rdm=True)
        worst = 0.0
        for b in range(L - 1):
            worst = max(worst, np.max(np.abs(rho[b] - _lightcone_rdm(L, hs, G, w["spinors"], n, b))))
        say(f"L=34 light-cone rdm worst {worst:.3e}, |N-1| {abs(N - 1):.3e}")
        assert worst < 2e-6
        assert abs(N - 1) < 1e-5
    finally:
        del psi
        torch.cuda.empty_cache()


def test_L33_complex128_in_place_lightcone_rdms():
    """The largest complex128 chain (L = 33, 128 GiB in place): bond density
    matrices after 2 periods against the oracle on light-cone subchains,
    every bond, to FP64 rounding."""
    L, n = 33, 2
    free, total = torch.cuda.mem_get_info()
    if free < (1 << L) * 16 + (8 << 30):
        pytest.skip(f"needs 136 GiB of free device memory, {free / 2**30:.0f} GiB free")
    say(f"case: L=33 complex128 light cone n={n}")
    w, hs = _model(L)
    G = O.floquet_gates(hs, w["T"])
    ctx = fl.fl_create(L, "c128")
    fl.fl_set_bonds(ctx, fl.fl_xyz_bonds(L, w["J"], w["fields"]), w["T"])
    psi = fl.new_state(ctx)
    try:
        fl.fl_init_state(ctx, psi, w["spinors"])
        fl.fl_apply_period(ctx, psi, n)
        E, N, rho = fl.fl_expect_energy(ctx, psi, rdm=True)
        worst = 0.0
        for b in range(L - 1):
            worst = max(worst, np.max(np.abs(rho[b] - _lightcone_rdm(L, hs, G, w["spinors"], n, b))))
        say(f"L=33 complex128 light-cone rdm worst {worst:.3e}, |N-1| {abs(N - 1):.3e}")
        assert worst < 1e-12
        assert abs(N - 1) < 1e-12
    finally:
        del psi
        torch.cuda.empty_cache()


@pytest.mark.parametrize("n", [5, 10, 16])
def test_L30_swap_point_and_ising_closed_forms(n):
    """Closed forms at full size: the SWAP point permutes the spinors (pins
    layer order, bit order and tile mapping); the diagonal chain conserves E.
    n = 10 and 16 run the benchmark's own plans (its 10-period step and its
    16-period sweep block)."""
    L = 30
    say(f"case: L=30 swap/ising n={n}")
    w = fin.xyz_workload(L, seed=5)
    ctx = fl.fl_create(L, "c64")
    J = np.full_like(w["J"], 2 * np.pi)
    f0 = np.zeros_like(w["fields"])
    fl.fl_set_bonds(ctx, fl.fl_xyz_bonds(L, J, f0), 0.25)
    psi = fl.new_state(ctx)
    fl.fl_init_state(ctx, psi, w["spinors"])
    fl.fl_apply_period(ctx, psi, n)
    order = list(range(L))
    for _ in range(n):
        for parity in (1, 0):
            for b in range(parity, L - 1, 2):
                order[b], order[b + 1] = order[b + 1], order[b]
    phase = np.exp(-1j * np.pi / 4 * (L - 1) * n)
    rng = np.random.default_rng(0)
    xs = rng.integers(0, 1 << L, 4096)
    got = psi[torch.from_numpy(xs).cuda()].cpu().numpy().astype(np.complex128)
    sp = [w["spinors"][order[j]] for j in range(L)]
    ref = np.array([phase * np.prod([sp[j][(x >> (L - 1 - j)) & 1] for j in range(L)]) for x in xs])
    assert np.max(np.abs(got - ref)) < 2e-6
    # diagonal chain: E conserved
    J2 = w["J"].copy(); J2[:, :2] = 0
    f2 = w["fields"].copy(); f2[:, :2] = 0
    fl.fl_set_bonds(ctx, fl.fl_xyz_bonds(L, J2, f2), 0.25)
    fl.fl_init_state(ctx, psi, w["spinors"])
    E0, N0 = fl.fl_expect_energy(ctx, psi)
    fl.fl_apply_period(ctx, psi, 20)
    E1, N1 = fl.fl_expect_energy(ctx, psi)
    assert abs(E0 - E1) < 1e-5 * L and abs(N1 - 1) < 1e-5
    del psi
    torch.cuda.empty_cache()


def test_L30_echo_fp32():
    """U_F^dagger^n U_F^n psi0 = psi0 at full size (Sec. V echo)."""
    L, n = 30, 10
    say("case: L=30 echo")
    w, hs = _model(L)
    ctx = fl.fl_create(L, "c64")
    fl.fl_set_bonds(ctx, fl.fl_xyz_bonds(L, w["J"], w["fields"]), w["T"])
    psi = fl.new_state(ctx)
    psi0 = fl.new_state(ctx)
    fl.fl_init_state(ctx, psi0, w["spinors"])
    psi.copy_(psi0)
    fl.fl_apply_period(ctx, psi, n)
    fl.fl_apply_period(ctx, psi, n, dagger=True)
    ov, n0, n1 = fl.fl_overlap(ctx, psi0, psi)
    say(f"L=30 echo overlap error {abs(1 - ov):.3e}")
    assert abs(1 - ov) < 1e-5
    del psi, psi0
    torch.cuda.empty_cache()


# ----------------------------------------------------------------- gradient

@pytest.mark.parametrize("L,n,K", [(2, 3, 0), (5, 4, 2), (10, 20, 5), (13, 8, 4), (14, 6, 3), (16, 6, 3)])
def test_gradient_fp64_matches_oracle_adjoint(L, n, K):
    say(f"case: grad fp64 L={L} n={n} K={K}")
    w, hs = _model(L, seed=31)
    G = O.floquet_gates(hs, w["T"])
    gens = O.xyz_coupling_generators(L)
    psi0 = O.product_state(w["spinors"])
    ref, Eref = O.adjoint_gradient(L, hs, gens, w["T"], psi0, n)
    ctx = fl.fl_create(L, "c128")
    fl.fl_set_bonds(ctx, hs, w["T"])
    psi = fl.new_state(ctx)
    fl.fl_init_state(ctx, psi, w["spinors"])
    ck = []
    if K:
        for _ in range(n // K):
            ck.append(psi.clone())
            fl.fl_apply_period(ctx, psi, K)
    else:
        fl.fl_apply_period(ctx, psi, n)
    lam = torch.empty_like(psi)
    g = fl.fl_grad(ctx, psi, ck, n, K, gens, lam)
    err = np.max(np.abs(g - ref)) / max(1.0, np.max(np.abs(ref)))
    say(f"grad fp64 L={L}: rel err {err:.3e}")
    assert err < 1e-10


def test_gradient_fp32_L12_close_to_fp64():
    L, n, K = 12, 40, 10
    say("case: grad fp32 L=12")
    w, hs = _model(L, seed=37)
    gens = O.xyz_coupling_generators(L)
    ref, _ = O.adjoint_gradient(L, hs, gens, w["T"], O.product_state(w["spinors"]), n)
    ctx = fl.fl_create(L, "c64")
    fl.fl_set_bonds(ctx, hs, w["T"])
    psi = fl.new_state(ctx)
    fl.fl_init_state(ctx, psi, w["spinors"])
    ck = []
    for _ in range(n // K):
        ck.append(psi.clone())
        fl.fl_apply_period(ctx, psi, K)
    g = fl.fl_grad(ctx, psi, ck, n, K, gens, torch.empty_like(psi))
    err = np.max(np.abs(g - ref)) / np.max(np.abs(ref))
    say(f"grad fp32 L=12: rel err {err:.3e}")
    assert err < 1e-4


def test_gradient_fp32_L16_close_to_fp64():
    # 12-bit tiles with first and last register groups moved straight
    # between HBM and registers as well as through LDS
    L, n, K = 16, 12, 4
    say("case: grad fp32 L=16")
    w, hs = _model(L, seed=43)
    gens = O.xyz_coupling_generators(L)
    ref, _ = O.adjoint_gradient(L, hs, gens, w["T"], O.product_state(w["spinors"]), n)
    ctx = fl.fl_create(L, "c64")
    fl.fl_set_bonds(ctx, hs, w["T"])
    psi = fl.new_state(ctx)
    fl.fl_init_state(ctx, psi, w["spinors"])
    ck = []
    for _ in range(n // K):
        ck.append(psi.clone())
        fl.fl_apply_period(ctx, psi, K)
    g = fl.fl_grad(ctx, psi, ck, n, K, gens, torch.empty_like(psi))
    err = np.max(np.abs(g - ref)) / np.max(np.abs(ref))
    say(f"grad fp32 L=16: rel err {err:.3e}")
    assert err < 1e-4


def test_gradient_fp32_L24_close_to_fp64_gpu():
    # 4096 tiles of 12 bits: every workgroup of the complex64 reverse pass
    # runs several tiles and copies the next one into LDS during the last
    # register group; the complex128 reverse pass (the reference here) has
    # no such copies.  Both start from the same product state.
    L, n, K = 24, 8, 4
    say("case: grad fp32 vs fp64 L=24")
    w, hs = _model(L, seed=47)
    gens = O.xyz_coupling_generators(L)
    out = {}
    for dt in ("c128", "c64"):
        ctx = fl.fl_create(L, dt)
        fl.fl_set_bonds(ctx, hs, w["T"])
        psi = fl.new_state(ctx)
        fl.fl_init_state(ctx, psi, w["spinors"])
        ck = []
        for _ in range(n // K):
            ck.append(psi.clone())
            fl.fl_apply_period(ctx, psi, K)
        out[dt] = fl.fl_grad(ctx, psi, ck, n, K, gens, torch.empty_like(psi))
        del psi, ck
        fl.fl_destroy(ctx)
        torch.cuda.empty_cache()
    err = np.max(np.abs(out["c64"] - out["c128"])) / np.max(np.abs(out["c128"]))
    say(f"grad fp32 vs fp64 L=24: rel err {err:.3e}")
    assert err < 1e-4


def test_autograd_function_matches_oracle():
    L, n, K = 8, 12, 4
    w, hs = _model(L, seed=41)
    eng = fl.FloquetEngine(L, "c128")
    J = torch.tensor(w["J"], dtype=torch.float64, requires_grad=True)
    T = torch.tensor(w["T"], dtype=torch.float64, requires_grad=True)
    E = fl.FloquetEnergy.apply(J, T, eng, w["fields"], w["spinors"], n, K)
    E.backward()
    ref, Eref = O.adjoint_gradient(L, hs, O.xyz_coupling_generators(L), w["T"],
                                   O.product_state(w["spinors"]), n)
    assert abs(E.item() - Eref) < 1e-12
    assert np.max(np.abs(J.grad.numpy().reshape(-1) - ref[:-1])) < 1e-10
    assert abs(T.grad.item() - ref[-1]) < 1e-10


# ----------------------------------------------------------------- measurement probe

@pytest.mark.parametrize("name", ["flp_fma_loop", "flp_fma_loop_v"])
def test_fma_probe_computes_its_recurrence(name):
    """The FMA-loop probes behind the bench's measured ceilings run the
    recurrence x <- 0.999 x + 0.001 they state (closed form in FP64)."""
    import ctypes
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2111_08044_amd", "libflprobe.so")
    lib = ctypes.CDLL(path)
    f = getattr(lib, name)
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    blocks, iters = 3, 500
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    assert f(out.data_ptr(), blocks, iters, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)) == 0
    torch.cuda.synchronize()
    a, b = np.float64(np.float32(0.999)), np.float64(np.float32(1e-3))
    t = np.arange(256, dtype=np.float64)
    x0 = np.float32(t * 1e-3)[None, :].astype(np.float64) + np.arange(16, dtype=np.float64)[:, None]
    ref = (a ** iters * x0 + b * (1 - a ** iters) / (1 - a)).sum(axis=0)
    got = out.cpu().numpy().reshape(blocks, 256)
    assert np.max(np.abs(got - ref[None, :]) / np.abs(ref)[None, :]) < 1e-4


# ----------------------------------------------------------------- degenerate depth

@pytest.mark.parametrize("dtype,variant", [("c64", "plain"), ("c128", "plain"), ("c64", "dense4_fp32")])
def test_zero_periods_is_the_identity_and_gradient_is_explicit(dtype, variant):
    """n = 0: fl_apply_period leaves the state bit-identical; the gradient
    then has only its explicit terms (Eq. (10) at t = 0), dE/dT = 0 (also
    through the window form's replay, which then runs no pass)."""
    L = 14
    say(f"case: zero periods {dtype} {variant} L={L}")
    w, hs = _model(L, seed=53)
    ctx = fl.fl_create(L, dtype, variant)
    fl.fl_set_bonds(ctx, hs, w["T"])
    psi = fl.new_state(ctx)
    fl.fl_init_state(ctx, psi, w["spinors"])
    fl.fl_apply_period(ctx, psi, 3)
    before = psi.clone()
    fl.fl_apply_period(ctx, psi, 0)
    fl.fl_apply_period(ctx, psi, 0, dagger=True)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(psi), torch.view_as_real(before))
    gens = O.xyz_coupling_generators(L)
    g = fl.fl_grad(ctx, psi, [], 0, 0, gens, torch.empty_like(psi))
    ref, _ = O.adjoint_gradient(L, hs, gens, w["T"], psi.cpu().numpy().astype(np.complex128), 0)
    tol = 1e-10 if dtype == "c128" else 1e-5
    assert abs(g[-1]) < tol * max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(g - ref)) < tol * max(1.0, np.max(np.abs(ref)))


# ----------------------------------------------------------------- ABI errors

def test_abi_error_paths_launch_nothing():
    L = 10
    ctx = fl.fl_create(L, "c64")
    psi = fl.new_state(ctx)
    with pytest.raises(fl.FloquetError) as e:
        fl.fl_apply_period(ctx, psi, 1)          # no bonds yet
    assert e.value.code == -4
    w, hs = _model(L)
    bad = hs.copy()
    bad[2, 0, 1] += 0.5                          # not Hermitian
    with pytest.raises(fl.FloquetError) as e:
        fl.fl_set_bonds(ctx, bad, 0.25)
    assert e.value.code == -1
    with pytest.raises(fl.FloquetError):
        fl.fl_set_bonds(ctx, hs, -1.0)
    fl.fl_set_bonds(ctx, hs, 0.25)
    lib = fl.lib()
    import ctypes as C
    assert lib.fl_apply_period(ctx.handle, C.c_void_p(psi.data_ptr()), -1, 0) == -1
    assert lib.fl_apply_period(ctx.handle, C.c_void_p(psi.data_ptr() + 8), 1, 0) == -1   # misaligned
    host = np.zeros(1 << L, dtype=np.complex64)
    assert lib.fl_apply_period(ctx.handle, C.c_void_p(host.ctypes.data), 1, 0) == -1      # host memory
    assert lib.fl_apply_period(ctx.handle, None, 1, 0) == -1
    with pytest.raises(fl.FloquetError):
        fl.fl_create(35, "c64")
    with pytest.raises(fl.FloquetError):
        fl.fl_create(34, "c128")
    lam = torch.empty_like(psi)
    with pytest.raises(fl.FloquetError):
        fl.fl_grad(ctx, psi, [psi.clone()], 10, 3, O.xyz_coupling_generators(L), lam)   # n % K != 0


# ------------------------------------------------- dense 6-qubit windows (MFMA)

# Per window application, relative L2 error of the state: FP32 MFMA rounds the
# window matrix and the products to FP32 (a few 2^-24 per entry, summed over
# 128 terms for 6-qubit windows, 32 for 4-qubit windows); split-BF16x3 keeps
# hi*hi + hi*lo + lo*hi of 8-bit splits, so the dropped lo*lo term and the
# split residuals are ~3 * 2^-17 relative.
DENSE_PER_WINDOW = {"dense6_fp32": 2e-6, "dense6_bf16x3": 4e-5, "dense4_fp32": 1e-6}
DENSE_PLAN_KIND = {"dense6_fp32": 4, "dense6_bf16x3": 4, "dense4_fp32": 5}


def _windows(L, n, dagger=False, variant="dense6_fp32"):
    from tests import plan_tools as pt
    _, _, _, passes = pt.parse_plan(fl.fl_plan_query(L, "c64", DENSE_PLAN_KIND[variant], n, dagger))
    return sum(len(g) for _, _, g in passes)


@pytest.mark.parametrize("variant,L", [(v, L) for v in ("dense6_fp32", "dense6_bf16x3") for L in (11, 12, 13, 14, 16)]
                         + [("dense4_fp32", L) for L in (13, 14, 16)])
def test_dense_windows_against_oracle(variant, L):
    say(f"case: dense {variant} L={L}")
    w, hs = _model(L, seed=200 + L)
    G = O.floquet_gates(hs, w["T"])
    ctx = fl.fl_create(L, "c64", variant)
    fl.fl_set_gates(ctx, G, hs, w["T"])
    psi = _gpu_state(ctx)
    fl.fl_init_state(ctx, psi, w["spinors"])
    ref = O.product_state(w["spinors"])
    napp = 0
    for n in (1, 7, 17):
        fl.fl_apply_period(ctx, psi, n)
        ref = O.evolve(ref, L, G, n)
        napp += _windows(L, n, False, variant)
        err = np.linalg.norm(psi.cpu().numpy().astype(np.complex128) - ref)
        say(f"  n={n} windows={napp} L2 err {err:.3e}")
        assert err < napp * DENSE_PER_WINDOW[variant], (n, err)
    fl.fl_apply_period(ctx, psi, 25, dagger=True)
    napp += _windows(L, 25, True, variant)
    err = np.linalg.norm(psi.cpu().numpy().astype(np.complex128) - O.product_state(w["spinors"]))
    assert err < napp * DENSE_PER_WINDOW[variant], err


@pytest.mark.parametrize("variant", ["dense6_fp32", "dense6_bf16x3", "dense4_fp32"])
def test_dense_L30_lightcone_rdms(variant):
    """L = 30 through the dense windows: bond density matrices after 3 periods
    against the oracle on light-cone subchains."""
    L, n = 30, 3
    say(f"case: dense {variant} L=30 light cone")
    w, hs = _model(L)
    G = O.floquet_gates(hs, w["T"])
    ctx = fl.fl_create(L, "c64", variant)
    fl.fl_set_bonds(ctx, fl.fl_xyz_bonds(L, w["J"], w["fields"]), w["T"])
    psi = fl.new_state(ctx)
    fl.fl_init_state(ctx, psi, w["spinors"])
    fl.fl_apply_period(ctx, psi, n)
    E, N, rho = fl.fl_expect_energy(ctx, psi, rdm=True)
    worst = 0.0
    for b in (0, 5, 12, 13, 20, 28):
        worst = max(worst, np.max(np.abs(rho[b] - _lightcone_rdm(L, hs, G, w["spinors"], n, b))))
    napp = _windows(L, n, False, variant)
    say(f"dense {variant} L=30: worst rdm err {worst:.3e} over {napp} windows, |N-1| {abs(N - 1):.3e}")
    assert worst < 4 * napp * DENSE_PER_WINDOW[variant]
    del psi
    torch.cuda.empty_cache()
