"""MI355X (gfx950) Floquet brickwork engine: Python binding of libfloquet.so.

The functions below carry the names of the C ABI (include/floquet.h) and only
marshal arguments: torch tensors supply device memory and the current HIP
stream, NumPy arrays supply host parameters.  Every step of the computation
runs in the library's kernels.

    ctx = fl_create(L, "c64")
    fl_set_bonds(ctx, h, T)                      # h: (L-1, 4, 4) complex
    psi = new_state(ctx)                         # torch tensor on the GPU
    fl_init_state(ctx, psi, spinors)             # spinors: (L, 2) complex
    fl_apply_period(ctx, psi, n)
    E, N = fl_expect_energy(ctx, psi)
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _native
from ._native import (FL_C64, FL_C128, FL_PLAIN, FL_DENSE6_FP32, FL_DENSE6_BF16X3, FL_DENSE4_FP32,  # noqa: F401
                      FloquetError, check, lib)

__all__ = [
    "fl_create", "fl_destroy", "fl_set_bonds", "fl_set_gates", "fl_init_state", "fl_init_pairs", "fl_apply_period",
    "fl_expect_energy", "fl_expect_energy_noalloc", "fl_energy_spread", "fl_overlap", "fl_grad_workspace_bytes", "fl_grad",
    "fl_last_error", "fl_xyz_bonds", "fl_xyz_generators", "fl_host_gates", "fl_host_gate_derivative",
    "fl_host_ground_states",
    "fl_plan_query", "fl_tile_map", "fl_host_window_matrix", "fl_host_window_overlaps", "Context", "new_state", "FloquetEngine", "FloquetEnergy",
    "thermalization_rate", "fit_exponential_rate",
]

_DTYPES = {"c64": FL_C64, "c128": FL_C128}
_VARIANTS = {"plain": FL_PLAIN, "dense6_fp32": FL_DENSE6_FP32, "dense6_bf16x3": FL_DENSE6_BF16X3,
             "dense4_fp32": FL_DENSE4_FP32}


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _c16(a, shape) -> np.ndarray:
    """complex array -> contiguous float64 (re, im) interleaved."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128).reshape(shape))
    return a.view(np.float64)


def _torch():
    import torch
    return torch


class Context:
    """Owning handle of an fl_ctx."""

    def __init__(self, handle, L, dtype, variant):
        self.handle = handle
        self.L = L
        self.dtype = dtype
        self.variant = variant

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h:
            try:
                lib().fl_destroy(h)
            except Exception:
                pass

    @property
    def torch_dtype(self):
        torch = _torch()
        return torch.complex64 if self.dtype == FL_C64 else torch.complex128


def _stream(ctx: Context):
    torch = _torch()
    check(lib().fl_set_stream(ctx.handle, C.c_void_p(torch.cuda.current_stream().cuda_stream)))


def _state_ptr(ctx: Context, t, name="psi"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP torch tensor")
    want = ctx.torch_dtype
    if t.dtype != want or t.numel() != (1 << ctx.L) or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {want} tensor of 2^{ctx.L} elements")
    return C.c_void_p(t.data_ptr())


def fl_last_error() -> str:
    return lib().fl_last_error().decode(errors="replace")


def fl_create(L: int, dtype="c64", variant="plain") -> Context:
    dt = _DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    va = _VARIANTS[variant] if isinstance(variant, str) else int(variant)
    h = C.c_void_p()
    torch = _torch()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream) if torch.cuda.is_available() else None
    check(lib().fl_create(C.byref(h), int(L), dt, va, stream))
    return Context(h, int(L), dt, va)


def fl_destroy(ctx: Context):
    h, ctx.handle = ctx.handle, None
    if h:
        check(lib().fl_destroy(h))


def new_state(ctx: Context):
    torch = _torch()
    return torch.empty(1 << ctx.L, dtype=ctx.torch_dtype, device="cuda")


def fl_set_bonds(ctx: Context, h, T: float):
    hb = _c16(h, (ctx.L - 1, 4, 4))
    _stream(ctx)
    check(lib().fl_set_bonds(ctx.handle, _dp(hb), float(T)))


def fl_set_gates(ctx: Context, G, h=None, T: float = 0.0):
    Gb = _c16(G, (ctx.L - 1, 4, 4))
    hb = _c16(h, (ctx.L - 1, 4, 4)) if h is not None else None
    _stream(ctx)
    check(lib().fl_set_gates(ctx.handle, _dp(Gb), _dp(hb) if hb is not None else None, float(T)))


def fl_init_state(ctx: Context, psi, spinors):
    s = _c16(spinors, (ctx.L, 2))
    _stream(ctx)
    check(lib().fl_init_state(ctx.handle, _state_ptr(ctx, psi), _dp(s)))


def fl_init_pairs(ctx: Context, psi, pairs, tail=None):
    """psi <- prod_m pairs[m] on sites (2m, 2m+1) (and tail on the last site for odd L)."""
    p = _c16(pairs, (ctx.L // 2, 4))
    t = _c16(tail, (2,)) if tail is not None else None
    _stream(ctx)
    check(lib().fl_init_pairs(ctx.handle, _state_ptr(ctx, psi), _dp(p), _dp(t) if t is not None else None))


def fl_apply_period(ctx: Context, psi, n: int, dagger: bool = False):
    _stream(ctx)
    check(lib().fl_apply_period(ctx.handle, _state_ptr(ctx, psi), int(n), 1 if dagger else 0))


def fl_expect_energy(ctx: Context, psi, rdm: bool = False):
    """(<H0>, <psi|psi>) and, with rdm=True, the (L-1, 4, 4) bond density matrices."""
    out = np.zeros(2)
    r = np.zeros((ctx.L - 1, 4, 4), dtype=np.complex128) if rdm else None
    _stream(ctx)
    check(lib().fl_expect_energy(ctx.handle, _state_ptr(ctx, psi), _dp(out),
                                 _dp(r.view(np.float64)) if rdm else None))
    return (out[0], out[1], r) if rdm else (out[0], out[1])


def fl_expect_energy_noalloc(ctx: Context, psi, out, rdm=None):
    """Energy readout into device tensors, no allocation, no host wait:
    out (2 float64 on the GPU) <- (<H0>, <psi|psi>); rdm (None or (L-1)*32
    float64 on the GPU) <- the bond density matrices."""
    torch = _torch()
    for name, t, n in (("out", out, 2), ("rdm", rdm, (ctx.L - 1) * 32)):
        if t is None and name == "rdm":
            continue
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or t.numel() != n \
                or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 GPU tensor of {n} elements")
    _stream(ctx)
    check(lib().fl_expect_energy_noalloc(ctx.handle, _state_ptr(ctx, psi), C.c_void_p(out.data_ptr()),
                                         C.c_void_p(rdm.data_ptr()) if rdm is not None else None))


def fl_energy_spread(ctx: Context, psi, ws):
    """(<H0>, <H0^2>, <psi|psi>), un-normalised; ws receives H0 psi."""
    out = np.zeros(3)
    _stream(ctx)
    check(lib().fl_energy_spread(ctx.handle, _state_ptr(ctx, psi), _state_ptr(ctx, ws, "ws"), _dp(out)))
    return out[0], out[1], out[2]


def fl_overlap(ctx: Context, phi, psi):
    """(<phi|psi>, <phi|phi>, <psi|psi>) for complex64/complex128 tensors."""
    torch = _torch()
    for t in (phi, psi):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.numel() != (1 << ctx.L) or not t.is_contiguous():
            raise ValueError("phi/psi must be contiguous GPU tensors of 2^L elements")
    dt = {torch.complex64: FL_C64, torch.complex128: FL_C128}
    out = np.zeros(4)
    _stream(ctx)
    check(lib().fl_overlap(ctx.handle, C.c_void_p(phi.data_ptr()), dt[phi.dtype], C.c_void_p(psi.data_ptr()),
                           dt[psi.dtype], _dp(out)))
    return complex(out[0], out[1]), out[2], out[3]


def fl_grad_workspace_bytes(ctx: Context) -> int:
    r = lib().fl_grad_workspace_bytes(ctx.handle)
    if r < 0:
        check(int(r))
    return int(r)


def fl_grad(ctx: Context, psi_n, ckpts, n: int, K: int, gens, lam_ws):
    """Gradient of <psi_n|H0|psi_n>: array of (L-1)*P + 1 values (last: d/dT)."""
    gens = np.asarray(gens)
    P = gens.shape[1]
    g = _c16(gens, (ctx.L - 1, P, 4, 4))
    ptrs = None
    if ckpts:
        arr = (C.c_void_p * len(ckpts))(*[_state_ptr(ctx, t, "ckpt").value for t in ckpts])
        ptrs = C.cast(arr, C.POINTER(C.c_void_p))
    out = np.zeros((ctx.L - 1) * P + 1)
    _stream(ctx)
    check(lib().fl_grad(ctx.handle, _state_ptr(ctx, psi_n, "psi_n"), ptrs, int(n), int(K), _dp(g), int(P),
                        _state_ptr(ctx, lam_ws, "lambda_ws"), _dp(out)))
    return out


# ----------------------------------------------------------------- host helpers

def fl_xyz_bonds(L: int, J, fields) -> np.ndarray:
    Jb = np.ascontiguousarray(np.asarray(J, dtype=np.float64).reshape(L - 1, 3))
    fb = np.ascontiguousarray(np.asarray(fields, dtype=np.float64).reshape(L, 3))
    out = np.zeros((L - 1, 4, 4), dtype=np.complex128)
    check(lib().fl_xyz_bonds(int(L), _dp(Jb), _dp(fb), _dp(out.view(np.float64))))
    return out


def fl_xyz_generators(L: int) -> np.ndarray:
    out = np.zeros((L - 1, 3, 4, 4), dtype=np.complex128)
    check(lib().fl_xyz_generators(int(L), _dp(out.view(np.float64))))
    return out


def fl_host_gates(h, T: float) -> np.ndarray:
    h = np.asarray(h, dtype=np.complex128)
    nb = h.shape[0]
    hb = _c16(h, (nb, 4, 4))
    out = np.zeros((nb, 4, 4), dtype=np.complex128)
    check(lib().fl_host_gates(nb, _dp(hb), float(T), _dp(out.view(np.float64))))
    return out


def fl_host_gate_derivative(h, gen, T: float) -> np.ndarray:
    hb = _c16(h, (4, 4))
    gb = _c16(gen, (4, 4))
    out = np.zeros((4, 4), dtype=np.complex128)
    check(lib().fl_host_gate_derivative(_dp(hb), _dp(gb), float(T), _dp(out.view(np.float64))))
    return out


def fl_host_ground_states(h):
    """(g, e0): lowest eigenvectors (n, 4) and eigenvalues (n,) of n 4x4 Hermitian matrices."""
    h = np.asarray(h, dtype=np.complex128)
    n = h.reshape(-1, 4, 4).shape[0]
    hb = _c16(h, (n, 4, 4))
    g = np.zeros((n, 4), dtype=np.complex128)
    e = np.zeros(n)
    check(lib().fl_host_ground_states(n, _dp(hb), _dp(g.view(np.float64)), _dp(e)))
    return g, e


def fl_host_window_matrix(G, pos, mode=None):
    """(U, fragments) of a dense window: U = E(op_n-1)...E(op_0) and, for mode
    0/1 (6-bit window, U 64x64), the MFMA fragments as raw bytes (mode 0:
    64 KiB FP32, mode 1: 32 KiB of bf16 hi/lo (Re, Im) pairs); mode 2: 4-bit
    window, U 16x16, 4 KiB of FP32 fragments."""
    G = np.asarray(G, dtype=np.complex128)
    n = G.shape[0]
    Gb = _c16(G, (n, 4, 4))
    p = np.ascontiguousarray(np.asarray(pos, dtype=np.int32))
    dim = 16 if mode == 2 else 64
    U = np.zeros((dim, dim), dtype=np.complex128)
    frag = (np.zeros({0: 65536, 1: 32768, 2: 4096}.get(int(mode), 65536), dtype=np.uint8)
            if mode is not None else None)
    check(lib().fl_host_window_matrix(_dp(Gb), p.ctypes.data_as(C.POINTER(C.c_int)), n,
                                      -1 if mode is None else int(mode), _dp(U.view(np.float64)),
                                      frag.ctypes.data_as(C.c_void_p) if frag is not None else None))
    return U, frag


def fl_host_window_overlaps(Q, G, pos) -> np.ndarray:
    """(nops, 16) overlap terms of a reverse register group from its 16x16
    window overlap Q and its ops (gates G (nops, 4, 4) on window bits pos)."""
    G = np.asarray(G, dtype=np.complex128).reshape(-1, 4, 4)
    n = G.shape[0]
    Qb = _c16(Q, (16, 16))
    Gb = _c16(G, (n, 4, 4))
    p = np.ascontiguousarray(np.asarray(pos, dtype=np.int32))
    out = np.zeros((n, 16))
    check(lib().fl_host_window_overlaps(_dp(Qb), _dp(Gb), p.ctypes.data_as(C.POINTER(C.c_int)), n, _dp(out)))
    return out


def fl_plan_query(L: int, dtype="c64", kind: int = 0, n: int = 1, dagger: bool = False) -> np.ndarray:
    dt = _DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    need = C.c_int64()
    check(lib().fl_plan_query(int(L), dt, int(kind), int(n), 1 if dagger else 0, None, 0, C.byref(need)))
    buf = np.zeros(need.value, dtype=np.int32)
    check(lib().fl_plan_query(int(L), dt, int(kind), int(n), 1 if dagger else 0,
                              buf.ctypes.data_as(C.POINTER(C.c_int32)), need.value, C.byref(need)))
    return buf


def fl_tile_map(L: int, dtype="c64", h: int = 0) -> np.ndarray:
    dt = _DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    out = np.zeros(1 << L, dtype=np.uint64)
    check(lib().fl_tile_map(int(L), dt, int(h), out.ctypes.data_as(C.POINTER(C.c_uint64))))
    return out


from .engine import FloquetEngine, FloquetEnergy, fit_exponential_rate, thermalization_rate  # noqa: E402
