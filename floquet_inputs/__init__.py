"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds none of the method's arithmetic: it only draws numbers.  It
produces the parameters of a workload (couplings, site fields, drive period)
and the single-site spinors of a random product initial state.  Both the CPU
oracle and the GPU path consume exactly these arrays.

Workload family (a synthetic stand-in for the paper's unpublished random
bond sample of Sec. III A): on every bond b = (b, b+1) of an open chain the bond
Hamiltonian has XYZ couplings (Jx, Jy, Jz) = (1.0, 0.8, 0.6) plus half of each
site's field vector.  Site fields are uniform in [-1, 1]^3.  The initial state
is a product of Haar-random single-qubit spinors (normalised complex Gaussian
2-vectors).  Sec. III A of the paper draws one long list of random terms once
and uses its first L-1 entries for an L-qubit chain; the same "first entries of
one long list" rule is used here so that chains of different L share their
parameters.

Draw order (fixed, so that every consumer sees the same numbers):
    rng = numpy.random.default_rng(seed)
    F = rng.uniform(-1, 1, (NMAX, 3))        site fields
    Z = rng.standard_normal((NMAX, 2, 2))    spinor real/imag parts
"""
from __future__ import annotations

import numpy as np

NMAX = 64
DEFAULT_SEED = 2111
DEFAULT_T = 0.25
DEFAULT_J = (1.0, 0.8, 0.6)


def xyz_workload(L: int, seed: int = DEFAULT_SEED, T: float = DEFAULT_T,
                 J=DEFAULT_J) -> dict:
    """Parameters of the XYZ-plus-fields Floquet chain of length L.

    Returns a dict with
      L        int
      T        float, drive period
      J        (L-1, 3) float64, per-bond couplings (Jx, Jy, Jz)
      fields   (L, 3) float64, per-site field vectors
      spinors  (L, 2) complex128, unit-norm single-site states
    """
    if not (2 <= L <= NMAX):
        raise ValueError(f"L must be in [2, {NMAX}], got {L}")
    rng = np.random.default_rng(seed)
    F = rng.uniform(-1.0, 1.0, (NMAX, 3))
    Z = rng.standard_normal((NMAX, 2, 2))
    s = Z[:L, :, 0] + 1j * Z[:L, :, 1]
    s = s / np.linalg.norm(s, axis=1, keepdims=True)
    Jarr = np.tile(np.asarray(J, dtype=np.float64), (L - 1, 1))
    return dict(L=L, T=float(T), J=Jarr, fields=F[:L].copy(), spinors=s)


def random_spinors(L: int, seed: int) -> np.ndarray:
    """(L, 2) complex128 Haar-random unit spinors from a given seed."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((L, 2, 2))
    s = Z[:, :, 0] + 1j * Z[:, :, 1]
    return s / np.linalg.norm(s, axis=1, keepdims=True)


def random_fields(L: int, seed: int) -> np.ndarray:
    """(L, 3) float64 site fields, uniform in [-1, 1]^3."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, (L, 3))


def gue_bond_sample(L: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    """(L-1, 4, 4) complex128 random Hermitian 4x4 matrices from the Gaussian
    unitary ensemble, shifted to be traceless and scaled to Frobenius norm
    sqrt(2) (the paper's model, Sec. III A).  One long list of NMAX terms is
    drawn and its first L-1 entries are returned."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((NMAX, 4, 4)) + 1j * rng.standard_normal((NMAX, 4, 4))
    H = (A + np.conj(np.swapaxes(A, 1, 2))) / 2.0
    tr = np.trace(H, axis1=1, axis2=2).real / 4.0
    H = H - tr[:, None, None] * np.eye(4)[None]
    nrm = np.sqrt(np.sum(np.abs(H) ** 2, axis=(1, 2)))
    H = H * (np.sqrt(2.0) / nrm)[:, None, None]
    return H[: L - 1].copy()


def random_state(L: int, seed: int) -> np.ndarray:
    """A random (unnormalised) complex128 state vector of 2^L amplitudes."""
    rng = np.random.default_rng(seed)
    n = 1 << L
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def random_unitaries(count: int, dim: int, seed: int) -> np.ndarray:
    """(count, dim, dim) complex128 Haar-random unitaries: QR of complex
    Gaussian matrices with the phases of R's diagonal moved into Q."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((count, dim, dim)) + 1j * rng.standard_normal((count, dim, dim))
    out = np.empty((count, dim, dim), dtype=np.complex128)
    for k in range(count):
        q, r = np.linalg.qr(Z[k])
        d = np.diag(r)
        out[k] = q * (d / np.abs(d))[None, :]
    return out
