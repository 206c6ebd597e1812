"""GPU parity at the benchmark's full size with distinct gates, the gradient at
its configured depth, the autograd wrapper's bookkeeping and the stream
contract of the C ABI (MI355X only; every call goes through the C ABI).

Full-size distinct-gate runs use circuits whose exact state the oracle can
still hold: inside a few windows of six bonds every bond carries its own
Haar-random two-qubit unitary, every other bond a product u_b (x) v_b of
single-qubit unitaries (all different).  The state then stays a product of
one 7-site state per window and single-site spinors, so every amplitude and
every bond density matrix of the 2^30-amplitude state is known exactly, while
a wrong gate index, a transposed gate, a wrong layer order or a wrong tile map
anywhere in the plan changes them.
"""
import sys

import numpy as np
import pytest

import floquet_inputs as fin
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2111_08044_amd as fl  # noqa: E402
from tests.windowed import WindowedCircuit  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _model(L, seed=fin.DEFAULT_SEED, T=0.25):
    w = fin.xyz_workload(L, seed=seed, T=T)
    return w, O.xyz_bond_hamiltonians(L, w["J"], w["fields"])


# Bond windows at L = 30 (bond b acts on bits L-2-b, L-1-b): the top bits,
# two mid-chain windows, and one across the low-bit boundaries (bits 1..7:
# bond 25 straddles bits 3 and 4, the edge between the complex64 sweep's 4
# contiguous low tile bits and its high window; bond 23 straddles bits 5 and
# 6, the same edge for the 6-low-bit tiles of the energy reduction).
L30_WINDOWS = [(0, 5), (7, 12), (14, 19), (22, 27)]


@pytest.mark.parametrize("n", [8, 10, 16])
def test_L30_distinct_gates_through_the_bench_plans(n):
    """L = 30 complex64, n = 10 (the benchmark step's plan), 16 (its
    sweep block) and 8: sampled amplitudes and every bond density matrix
    against the exact factorised state."""
    L = 30
    say(f"case: L=30 distinct gates n={n}")
    wc = WindowedCircuit(L, L30_WINDOWS, seed=900 + n)
    sp = fin.random_spinors(L, 901 + n)
    wins, sites = wc.evolve(sp, n)
    ctx = fl.fl_create(L, "c64")
    fl.fl_set_gates(ctx, wc.G)
    psi = fl.new_state(ctx)
    try:
        fl.fl_init_state(ctx, psi, sp)
        fl.fl_apply_period(ctx, psi, n)
        E, N, rho = fl.fl_expect_energy(ctx, psi, rdm=True)
        rng = np.random.default_rng(n)
        xs = rng.integers(0, 1 << L, 8192)
        got = psi[torch.from_numpy(xs).cuda()].cpu().numpy().astype(np.complex128)
        ref = wc.amplitudes(wins, sites, xs)
        amp_err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        worst = max(np.max(np.abs(rho[b] - wc.bond_rdm(wins, sites, b))) for b in range(L - 1))
        say(f"L=30 distinct gates n={n}: sampled amplitudes rel L2 {amp_err:.3e}, worst rdm {worst:.3e}, "
            f"|N-1| {abs(N - 1):.3e}")
        assert amp_err < 1e-5
        assert worst < 2e-6
        assert abs(N - 1) < 1e-5
    finally:
        del psi
        torch.cuda.empty_cache()


# ------------------------------------------------------ gradient at depth

@pytest.mark.parametrize("L", [14, 16])
def test_gradient_fp32_at_configured_depth_matches_oracle_adjoint(L):
    """complex64 fl_grad at the configured depth n = 200 with checkpoints
    every K = 50 periods (the G^dagger replay of Sec. V) against the FP64
    oracle adjoint: relative error <= 1e-3 of the largest component."""
    n, K = 200, 50
    say(f"case: grad fp32 L={L} n={n} K={K}")
    w, hs = _model(L, seed=61)
    gens = O.xyz_coupling_generators(L)
    ref, Eref = O.adjoint_gradient(L, hs, gens, w["T"], O.product_state(w["spinors"]), n)
    ctx = fl.fl_create(L, "c64")
    fl.fl_set_bonds(ctx, hs, w["T"])
    psi = fl.new_state(ctx)
    fl.fl_init_state(ctx, psi, w["spinors"])
    ck = []
    for _ in range(n // K):
        ck.append(psi.clone())
        fl.fl_apply_period(ctx, psi, K)
    E, N = fl.fl_expect_energy(ctx, psi)
    g = fl.fl_grad(ctx, psi, ck, n, K, gens, torch.empty_like(psi))
    err = np.max(np.abs(g - ref)) / np.max(np.abs(ref))
    say(f"grad fp32 L={L} n={n}: rel err {err:.3e}, |E-Eref|/L {abs(E - Eref) / L:.3e}")
    assert abs(E - Eref) / L < 1e-5
    assert err < 1e-3


def test_gradient_c4_config_fp32_against_fp64_gpu():
    """The adjoint workload itself: L = 24, n = 200, K = 50, complex64
    gradient of all 3(L-1) couplings and T against the complex128 GPU
    gradient (pinned to the oracle adjoint at 1e-10 by the FP64 tests):
    relative error <= 1e-3; E_n within 1e-5 per site."""
    L, n, K = 24, 200, 50
    say(f"case: grad C4 L={L} n={n} K={K}")
    w, hs = _model(L)
    gens = O.xyz_coupling_generators(L)
    out = {}
    for dt in ("c128", "c64"):
        ctx = fl.fl_create(L, dt)
        fl.fl_set_bonds(ctx, fl.fl_xyz_bonds(L, w["J"], w["fields"]), w["T"])
        psi = fl.new_state(ctx)
        fl.fl_init_state(ctx, psi, w["spinors"])
        ck = []
        for _ in range(n // K):
            ck.append(psi.clone())
            fl.fl_apply_period(ctx, psi, K)
        E, N = fl.fl_expect_energy(ctx, psi)
        out[dt] = (fl.fl_grad(ctx, psi, ck, n, K, gens, torch.empty_like(psi)), E / N)
        del psi, ck
        fl.fl_destroy(ctx)
        torch.cuda.empty_cache()
    g64, e64 = out["c128"]
    g32, e32 = out["c64"]
    err = np.max(np.abs(g32 - g64)) / np.max(np.abs(g64))
    say(f"grad C4: rel err {err:.3e} (max |g| {np.max(np.abs(g64)):.3e}), |dE|/L {abs(e32 - e64) / L:.3e}, "
        f"dE/dT {g32[-1]:.6f} vs {g64[-1]:.6f}")
    assert abs(e32 - e64) / L < 1e-5
    assert err < 1e-3


# ------------------------------------- gradient of the 4-qubit-window form

@pytest.mark.parametrize("L,n,K,tol", [(14, 200, 50, 1e-4), (16, 200, 50, 1e-3), (14, 50, 10, 1e-4),
                                       (16, 37, 0, 1e-4), (15, 21, 7, 1e-4)])
def test_gradient_dense4_matches_oracle_adjoint(L, n, K, tol):
    """The 4-qubit-window form (FP32 MFMA windows forward, their exact
    adjoints replayed on the matrix cores with the window-overlap terms)
    against the FP64 oracle adjoint: at the configured depth n = 200, K = 50,
    with many checkpoint resets (K = 10), with none (K = 0), and with
    segments that end in a partial plan block (K = 7).  Relative error of the
    largest component <= 1e-4.  At L = 16, n = 200 the gradient of this seed
    is small (largest component 0.59, against 10.7 at L = 14), so the same
    FP32 rounding (1e-4 to 2.5e-4 absolute, depending on the order of the
    sums that the tile geometry fixes; the plain form's error there ranges
    over 5e-5 to 1.7e-4 relative) reads as up to 4e-4 relative: there the
    bound is 1e-3.  (A replay with windows that are not the exact adjoints of
    the forward's FP32 matrices misses the 1e-4 bounds by an order of
    magnitude once checkpoints reset psi: 1.1e-3 at L = 14, n = 200, K = 50.)"""
    say(f"case: grad dense4 L={L} n={n} K={K}")
    w, hs = _model(L, seed=61)
    gens = O.xyz_coupling_generators(L)
    ref, Eref = O.adjoint_gradient(L, hs, gens, w["T"], O.product_state(w["spinors"]), n)
    ctx = fl.fl_create(L, "c64", "dense4_fp32")
    fl.fl_set_bonds(ctx, hs, w["T"])
    psi = fl.new_state(ctx)
    fl.fl_init_state(ctx, psi, w["spinors"])
    ck = []
    if K > 0:
        for _ in range(n // K):
            ck.append(psi.clone())
            fl.fl_apply_period(ctx, psi, K)
    else:
        fl.fl_apply_period(ctx, psi, n)
    E, N = fl.fl_expect_energy(ctx, psi)
    g = fl.fl_grad(ctx, psi, ck, n, K, gens, torch.empty_like(psi))
    err = np.max(np.abs(g - ref)) / np.max(np.abs(ref))
    say(f"grad dense4 L={L} n={n} K={K}: rel err {err:.3e} (dE/dT {g[-1]:.6f} vs {ref[-1]:.6f}), "
        f"|E-Eref|/L {abs(E - Eref) / L:.3e}")
    fl.fl_destroy(ctx)
    assert abs(E - Eref) / L < 1e-5
    assert err < tol


@pytest.mark.parametrize("variant,L", [("dense6_fp32", 14), ("dense6_bf16x3", 14), ("dense4_fp32", 13)])
def test_gradient_gate_by_gate_replay_of_window_forms_without_resets(variant, L):
    """The 6-qubit window forms (and the 4-qubit one on a single 13-bit
    tile) replay gate by gate, which is not the exact adjoint of their
    window matrices; without checkpoint resets (K = 0) the replay stays
    consistent and the gradient matches the oracle adjoint (relative error
    of the largest component <= 1e-4 at n = 50)."""
    n = 50
    say(f"case: grad {variant} L={L} n={n} K=0")
    w, hs = _model(L, seed=61)
    gens = O.xyz_coupling_generators(L)
    ref, Eref = O.adjoint_gradient(L, hs, gens, w["T"], O.product_state(w["spinors"]), n)
    ctx = fl.fl_create(L, "c64", variant)
    fl.fl_set_bonds(ctx, hs, w["T"])
    psi = fl.new_state(ctx)
    fl.fl_init_state(ctx, psi, w["spinors"])
    fl.fl_apply_period(ctx, psi, n)
    g = fl.fl_grad(ctx, psi, [], n, 0, gens, torch.empty_like(psi))
    err = np.max(np.abs(g - ref)) / np.max(np.abs(ref))
    say(f"grad {variant} L={L} n={n} K=0: rel err {err:.3e}")
    fl.fl_destroy(ctx)
    assert err < 1e-4


def test_gradient_c4_config_dense4_against_fp64_gpu():
    """The adjoint workload (L = 24, n = 200, K = 50) in the 4-qubit-window
    form against the complex128 GPU gradient: relative error <= 1e-4, E_n
    within 1e-5 per site."""
    L, n, K = 24, 200, 50
    say(f"case: grad C4 dense4 L={L} n={n} K={K}")
    w, hs = _model(L)
    gens = O.xyz_coupling_generators(L)
    out = {}
    for dt, va in (("c128", "plain"), ("c64", "dense4_fp32")):
        ctx = fl.fl_create(L, dt, va)
        fl.fl_set_bonds(ctx, fl.fl_xyz_bonds(L, w["J"], w["fields"]), w["T"])
        psi = fl.new_state(ctx)
        fl.fl_init_state(ctx, psi, w["spinors"])
        ck = []
        for _ in range(n // K):
            ck.append(psi.clone())
            fl.fl_apply_period(ctx, psi, K)
        E, N = fl.fl_expect_energy(ctx, psi)
        out[dt] = (fl.fl_grad(ctx, psi, ck, n, K, gens, torch.empty_like(psi)), E / N)
        del psi, ck
        fl.fl_destroy(ctx)
        torch.cuda.empty_cache()
    g64, e64 = out["c128"]
    g32, e32 = out["c64"]
    err = np.max(np.abs(g32 - g64)) / np.max(np.abs(g64))
    say(f"grad C4 dense4: rel err {err:.3e} (max |g| {np.max(np.abs(g64)):.3e}), |dE|/L {abs(e32 - e64) / L:.3e}, "
        f"dE/dT {g32[-1]:.6f} vs {g64[-1]:.6f}")
    assert abs(e32 - e64) / L < 1e-5
    assert err < 1e-4


def test_autograd_interleaved_forwards_use_their_own_couplings():
    """Two forwards on one engine with different couplings, then one
    backward through both: each gradient is the oracle's for its own J."""
    L, n, K = 8, 12, 4
    w, _ = _model(L, seed=71)
    eng = fl.FloquetEngine(L, "c128")
    J1 = torch.tensor(w["J"], dtype=torch.float64, requires_grad=True)
    J2 = torch.tensor(w["J"] * np.array([0.7, 1.3, -0.5]), dtype=torch.float64, requires_grad=True)
    T1 = torch.tensor(w["T"], dtype=torch.float64, requires_grad=True)
    T2 = torch.tensor(0.4, dtype=torch.float64, requires_grad=True)
    E1 = fl.FloquetEnergy.apply(J1, T1, eng, w["fields"], w["spinors"], n, K)
    E2 = fl.FloquetEnergy.apply(J2, T2, eng, w["fields"], w["spinors"], n, 0)
    (E1 + 2.0 * E2).backward()
    psi0 = O.product_state(w["spinors"])
    gens = O.xyz_coupling_generators(L)
    for J, T, E, scale in ((J1, T1, E1, 1.0), (J2, T2, E2, 2.0)):
        hs = O.xyz_bond_hamiltonians(L, J.detach().numpy(), w["fields"])
        ref, Eref = O.adjoint_gradient(L, hs, gens, T.item(), psi0, n)
        assert abs(E.item() - Eref) < 1e-12
        assert np.max(np.abs(J.grad.numpy().reshape(-1) - scale * ref[:-1])) < 1e-10
        assert abs(T.grad.item() - scale * ref[-1]) < 1e-10


# ------------------------------------------------------ stream contract

def test_uploads_and_init_are_ordered_on_a_side_stream():
    """On a non-default stream, with no host synchronisation in between:
    init, U_F(A)^n, set_bonds(B), U_F(B)^n, set_bonds(A) again and
    re-initialise a second state.  The gate upload for B must land after the
    A sweep has run and before the B sweep, and the asynchronous init must
    not race its table upload."""
    L, n = 18, 40
    say(f"case: side stream L={L} n={n}")
    wA, hA = _model(L, seed=81)
    wB, hB = _model(L, seed=82, T=0.31)
    GA, GB = O.floquet_gates(hA, wA["T"]), O.floquet_gates(hB, wB["T"])
    ref = O.evolve(O.evolve(O.product_state(wA["spinors"]), L, GA, n), L, GB, n)
    ref2 = O.evolve(O.product_state(wB["spinors"]), L, GA, 3)
    side = torch.cuda.Stream()
    ctx = fl.fl_create(L, "c128")
    with torch.cuda.stream(side):
        psi = torch.empty(1 << L, dtype=torch.complex128, device="cuda")
        psi2 = torch.empty(1 << L, dtype=torch.complex128, device="cuda")
        fl.fl_set_bonds(ctx, hA, wA["T"])
        fl.fl_init_state(ctx, psi, wA["spinors"])
        fl.fl_apply_period(ctx, psi, n)
        fl.fl_set_bonds(ctx, hB, wB["T"])
        fl.fl_apply_period(ctx, psi, n)
        fl.fl_set_bonds(ctx, hA, wA["T"])
        fl.fl_init_state(ctx, psi2, wB["spinors"])
        fl.fl_apply_period(ctx, psi2, 3)
    side.synchronize()
    err = np.linalg.norm(psi.cpu().numpy() - ref)
    err2 = np.linalg.norm(psi2.cpu().numpy() - ref2)
    say(f"side stream: L2 {err:.3e}, {err2:.3e}")
    assert err < 1e-11 and err2 < 1e-12


def test_set_gates_rejects_a_non_unitary_gate():
    L = 10
    w, hs = _model(L)
    G = O.floquet_gates(hs, w["T"])
    ctx = fl.fl_create(L, "c64")
    bad = G.copy()
    bad[4] *= 1.001
    with pytest.raises(fl.FloquetError) as e:
        fl.fl_set_gates(ctx, bad, hs, w["T"])
    assert e.value.code == -1
    fl.fl_set_gates(ctx, G, hs, w["T"])
