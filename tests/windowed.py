"""Exact reference for full-size circuits with distinct gates (test helper).

Inside a few windows of bonds every bond carries its own two-qubit unitary;
every other bond carries a product u_b (x) v_b of single-qubit unitaries.  The
state then stays a product of one small state per window and single-site
spinors, so the oracle's own gate application on those small factors gives
every amplitude and every bond density matrix of a chain far too long for the
oracle to hold whole.
"""
import numpy as np

import floquet_inputs as fin
import oracle as O

I2 = np.eye(2, dtype=np.complex128)


class WindowedCircuit:
    """Gates and exact evolution of a chain whose entangling gates sit only
    inside `windows` (inclusive bond ranges); every other bond is u (x) v."""

    def __init__(self, L, windows, seed):
        self.L = L
        self.windows = windows
        self.owner = [-1] * L
        for k, (b0, b1) in enumerate(windows):
            for j in range(b0, b1 + 2):
                assert self.owner[j] == -1, "windows must not share sites"
                self.owner[j] = k
        nent = sum(b1 - b0 + 1 for b0, b1 in windows)
        U4 = fin.random_unitaries(nent, 4, seed)
        U2 = fin.random_unitaries(2 * (L - 1), 2, seed + 1)
        self.G = np.zeros((L - 1, 4, 4), dtype=np.complex128)
        self.uv = {}
        k4 = 0
        for b in range(L - 1):
            if self.owner[b] >= 0 and self.owner[b] == self.owner[b + 1]:
                self.G[b] = U4[k4]
                k4 += 1
            else:
                u, v = U2[2 * b], U2[2 * b + 1]
                self.uv[b] = (u, v)
                self.G[b] = np.kron(u, v)

    def evolve(self, spinors, n):
        """(window states, site spinors) after n periods, gate by gate in the
        oracle's layer order (Eq. (4)); single-site factors act on a window
        state through the oracle's bond application."""
        L = self.L
        wins = [O.product_state(spinors[b0:b1 + 2]) for b0, b1 in self.windows]
        sites = [np.array(s, dtype=np.complex128) for s in spinors]

        def one_site(j, U):
            k = self.owner[j]
            if k < 0:
                sites[j] = U @ sites[j]
                return
            s0 = self.windows[k][0]
            Ls = self.windows[k][1] - s0 + 2
            jl = j - s0
            if jl < Ls - 1:
                wins[k] = O.apply_bond(wins[k], Ls, jl, np.kron(U, I2))
            else:
                wins[k] = O.apply_bond(wins[k], Ls, jl - 1, np.kron(I2, U))

        for _ in range(n):
            for layer in O.layer_bonds(L):
                for b in layer:
                    if b in self.uv:
                        one_site(b, self.uv[b][0])
                        one_site(b + 1, self.uv[b][1])
                    else:
                        k = self.owner[b]
                        b0, b1 = self.windows[k]
                        wins[k] = O.apply_bond(wins[k], b1 - b0 + 2, b - b0, self.G[b])
        return wins, sites

    def amplitudes(self, wins, sites, xs):
        L = self.L
        out = np.ones(len(xs), dtype=np.complex128)
        for k, (b0, b1) in enumerate(self.windows):
            Ls = b1 - b0 + 2
            last = b0 + Ls - 1
            out *= wins[k][(xs >> (L - 1 - last)) & ((1 << Ls) - 1)]
        for j in range(L):
            if self.owner[j] < 0:
                out *= sites[j][(xs >> (L - 1 - j)) & 1]
        return out

    def site_rdm(self, wins, sites, j):
        k = self.owner[j]
        if k < 0:
            return np.outer(sites[j], sites[j].conj())
        s0 = self.windows[k][0]
        Ls = self.windows[k][1] - s0 + 2
        v = wins[k].reshape(1 << (j - s0), 2, 1 << (Ls - (j - s0) - 1))
        return np.einsum("xiz,xjz->ij", v, v.conj())

    def bond_rdm(self, wins, sites, b):
        k = self.owner[b]
        if k >= 0 and k == self.owner[b + 1]:
            b0, b1 = self.windows[k]
            return O.bond_rdm(wins[k], b1 - b0 + 2, b - b0)
        return np.kron(self.site_rdm(wins, sites, b), self.site_rdm(wins, sites, b + 1))
