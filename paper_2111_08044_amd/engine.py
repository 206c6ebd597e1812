"""Convenience wrappers over the C ABI: an engine object and the
torch.autograd.Function whose backward is the library's adjoint pass."""
from __future__ import annotations

import numpy as np

from . import (fl_apply_period, fl_create, fl_energy_spread, fl_expect_energy, fl_grad, fl_host_ground_states,
               fl_init_pairs, fl_init_state, fl_overlap, fl_set_bonds, fl_xyz_bonds, fl_xyz_generators, new_state)


class FloquetEngine:
    """One chain length, one precision, one variant; states are torch tensors."""

    def __init__(self, L: int, dtype: str = "c64", variant: str = "plain"):
        self.L = L
        self.ctx = fl_create(L, dtype, variant)
        self.generation = 0   # bumped by every change of the gates

    def set_bonds(self, h, T: float):
        self.h = np.asarray(h, dtype=np.complex128).reshape(self.L - 1, 4, 4).copy()
        fl_set_bonds(self.ctx, self.h, T)
        self.generation += 1

    def set_paper_model(self, Hk, omega: float):
        """The paper's circuit (Sec. III A): gates exp(-i H_k T), T = 2 pi / omega,
        i.e. bond Hamiltonians h_b = 2 H_k for the half-period gate exp(-i (T/2) h_b).
        The energy observable is then H0 = 2 H-bar (H-bar = sum_k H_k)."""
        self.set_bonds(2.0 * np.asarray(Hk, dtype=np.complex128), 2.0 * np.pi / omega)

    def set_xyz(self, J, fields, T: float):
        self.set_bonds(fl_xyz_bonds(self.L, J, fields), T)

    def new_state(self):
        return new_state(self.ctx)

    def init(self, psi, spinors):
        fl_init_state(self.ctx, psi, spinors)

    def init_pairs(self, psi, pairs, tail=None):
        fl_init_pairs(self.ctx, psi, pairs, tail)

    def init_ground_pairs(self, psi, tail=None):
        """The paper's initial state (Sec. IV, Eq. (9)): the ground state of
        every odd-k term (0-indexed even bond b) on its two sites; for odd L
        the last site carries `tail`."""
        g, _ = fl_host_ground_states(self.h[0::2][: self.L // 2])
        fl_init_pairs(self.ctx, psi, g, tail)

    def step(self, psi, n: int = 1, dagger: bool = False):
        fl_apply_period(self.ctx, psi, n, dagger)

    def energy(self, psi):
        return fl_expect_energy(self.ctx, psi)

    def energy_density(self, psi) -> float:
        E, N = fl_expect_energy(self.ctx, psi)
        return E / (self.L * N)

    def energy_spread(self, psi, ws):
        """(sigma_E, <H0>, <H0^2>) of the normalised state (Sec. IV, Eq. (10)-(11))."""
        E, E2, N = fl_energy_spread(self.ctx, psi, ws)
        e, e2 = E / N, E2 / N
        return float(np.sqrt(max(e2 - e * e, 0.0))), e, e2

    def overlap(self, phi, psi):
        return fl_overlap(self.ctx, phi, psi)

    def run(self, psi, n: int, every: int):
        """Evolve n periods, recording (period, e, <H0>/L, N) every `every` periods."""
        rows = []
        E, N = self.energy(psi)
        rows.append((0, E / (self.L * N), E / self.L, N))
        t = 0
        while t < n:
            k = min(every, n - t)
            self.step(psi, k)
            t += k
            E, N = self.energy(psi)
            rows.append((t, E / (self.L * N), E / self.L, N))
        return rows


def thermalization_rate(t, E, k1: int = 1, k2: int = 2):
    """Heating rate of Sec. IV: Gamma = 1 / (t_k2 - t_k1), where t_k is the
    first time at which E(t) = E(0) exp(-k), E measured from the
    infinite-temperature value 0 (traceless bond terms).  Crossings are
    interpolated linearly between samples.  Returns (Gamma, t_k1, t_k2), with
    None entries when E(t) does not get that far."""
    t = np.asarray(t, dtype=float)
    r = np.asarray(E, dtype=float) / float(E[0])

    def crossing(k):
        lvl = np.exp(-k)
        below = np.nonzero(r <= lvl)[0]
        if below.size == 0 or below[0] == 0:
            return None
        i = below[0]
        return t[i - 1] + (r[i - 1] - lvl) / (r[i - 1] - r[i]) * (t[i] - t[i - 1])

    t1, t2 = crossing(k1), crossing(k2)
    if t1 is None or t2 is None or t2 <= t1:
        return None, t1, t2
    return 1.0 / (t2 - t1), t1, t2


def fit_exponential_rate(omegas, gammas):
    """(a, b) of the least-squares fit log Gamma = a omega + b (Sec. IV)."""
    a, b = np.polyfit(np.asarray(omegas, dtype=float), np.log(np.asarray(gammas, dtype=float)), 1)
    return float(a), float(b)


def _torch():
    import torch
    return torch


class FloquetEnergy:
    """E_n(J, T) = <psi_n|H0|psi_n> of the XYZ-plus-fields chain as a
    differentiable torch function of the couplings J (L-1, 3) and the period T.

    forward evolves on the GPU, storing the state every K periods (K = 0: no
    checkpoints); n must be a multiple of K.  backward runs the library's
    reverse pass (G^dagger replay from those checkpoints) with the couplings,
    fields and period its own forward used: if the engine's gates changed in
    between (another forward, set_bonds, set_xyz), they are installed again
    first.  Each forward supports one backward (the saved state is consumed).

        E = FloquetEnergy.apply(J, T, engine, fields, spinors, n, K)
    """

    @staticmethod
    def check_depth(n, K):
        """The checkpoint schedule of Sec. V's reverse replay: states at
        periods 0, K, ..., n - K, so K must divide n (K = 0: none)."""
        n, K = int(n), int(K)
        if n < 0 or K < 0:
            raise ValueError(f"n = {n} and K = {K} must be >= 0")
        if K > 0 and n % K != 0:
            raise ValueError(f"n = {n} is not a multiple of the checkpoint interval K = {K}")
        return n, K

    @staticmethod
    def _fn():
        torch = _torch()

        class _F(torch.autograd.Function):
            @staticmethod
            def forward(ctx, J, T, engine, fields, spinors, n, K):
                n, K = FloquetEnergy.check_depth(n, K)
                L = engine.L
                Jn = J.detach().cpu().numpy().astype(np.float64).copy()
                fn = np.array(fields, dtype=np.float64, copy=True)
                Tn = float(T)
                engine.set_xyz(Jn, fn, Tn)
                ctx.params = (Jn, fn, Tn)
                ctx.generation = engine.generation
                psi = engine.new_state()
                engine.init(psi, spinors)
                ckpts = []
                if K > 0:
                    for _ in range(n // K):
                        ckpts.append(psi.clone())
                        engine.step(psi, K)
                else:
                    engine.step(psi, n)
                E, _ = engine.energy(psi)
                ctx.engine, ctx.psi, ctx.ckpts, ctx.n, ctx.K, ctx.L = engine, psi, ckpts, n, K, L
                return torch.tensor(E, dtype=torch.float64)

            @staticmethod
            def backward(ctx, gE):
                eng = ctx.engine
                if ctx.psi is None:
                    raise RuntimeError("FloquetEnergy: backward ran twice on one forward (its saved state is consumed)")
                if eng.generation != ctx.generation:
                    eng.set_xyz(*ctx.params)
                lam = torch.empty_like(ctx.psi)
                g = fl_grad(eng.ctx, ctx.psi, ctx.ckpts, ctx.n, ctx.K, fl_xyz_generators(ctx.L), lam)
                ctx.psi = ctx.ckpts = None
                gJ = torch.from_numpy(g[:-1].reshape(ctx.L - 1, 3).copy()) * gE
                gT = torch.tensor(g[-1], dtype=torch.float64) * gE
                return gJ, gT, None, None, None, None, None

        return _F

    @classmethod
    def apply(cls, J, T, engine, fields, spinors, n, K):
        cls.check_depth(n, K)
        return cls._fn().apply(J, T, engine, fields, spinors, n, K)
