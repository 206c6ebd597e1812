"""fl_expect_energy_noalloc (static device scratch, no allocation) against
fl_expect_energy through the C ABI, on two calls in a row per precision, the
second on a smaller chain, so the second call finds the first one's contents
in the shared scratch."""
import ctypes as C
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


def _case(L, dtype, seed):
    w = fin.xyz_workload(L, seed=seed)
    hs = O.xyz_bond_hamiltonians(L, w["J"], w["fields"])
    ctx = fl.fl_create(L, dtype)
    fl.fl_set_bonds(ctx, hs, w["T"])
    psi = fl.new_state(ctx)
    psi.copy_(torch.from_numpy(fin.random_state(L, seed)).to(psi.dtype))
    fl.fl_apply_period(ctx, psi, 3)
    return ctx, psi


@pytest.mark.parametrize("dtype,Ls", [("c64", (22, 15)), ("c128", (18, 12)), ("c64", (14, 5))])
def test_noalloc_readout_matches_fl_expect_energy(dtype, Ls):
    for L in Ls:
        say(f"case: noalloc readout {dtype} L={L}")
        ctx, psi = _case(L, dtype, 300 + L)
        E, N, rho = fl.fl_expect_energy(ctx, psi, rdm=True)
        out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        rdm = torch.full(((L - 1) * 32,), float("nan"), dtype=torch.float64, device="cuda")
        # straight through the C ABI
        rc = fl.lib().fl_expect_energy_noalloc(ctx.handle, C.c_void_p(psi.data_ptr()), C.c_void_p(out.data_ptr()),
                                               C.c_void_p(rdm.data_ptr()))
        assert rc == 0, fl.fl_last_error()
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        r = rdm.cpu().numpy().view(np.complex128).reshape(L - 1, 4, 4)
        say(f"  E {o[0]:.15e} vs {E:.15e}, N {o[1]:.15e} vs {N:.15e}, rdm max diff {np.max(np.abs(r - rho)):.2e}")
        assert o[1] == N                          # the same kernels and order
        assert np.array_equal(r, rho)
        assert abs(o[0] - E) <= 1e-13 * L * N
        # without the density matrices, through the binding
        out2 = torch.zeros(2, dtype=torch.float64, device="cuda")
        fl.fl_expect_energy_noalloc(ctx, psi, out2)
        torch.cuda.synchronize()
        assert np.array_equal(out2.cpu().numpy(), o)
        del psi
        fl.fl_destroy(ctx)


def test_noalloc_readout_rejects_bad_outputs():
    ctx, psi = _case(12, "c64", 5)
    lib = fl.lib()
    host = np.zeros(2)
    assert lib.fl_expect_energy_noalloc(ctx.handle, C.c_void_p(psi.data_ptr()),
                                        C.c_void_p(host.ctypes.data), None) == -1
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    assert lib.fl_expect_energy_noalloc(ctx.handle, C.c_void_p(psi.data_ptr()),
                                        C.c_void_p(out.data_ptr() + 4), None) == -1
    assert lib.fl_expect_energy_noalloc(ctx.handle, C.c_void_p(psi.data_ptr()), None, None) == -1
    ctx2 = fl.fl_create(12, "c64")
    assert lib.fl_expect_energy_noalloc(ctx2.handle, C.c_void_p(psi.data_ptr()),
                                        C.c_void_p(out.data_ptr()), None) == -4   # no bonds yet
