"""Lattice geometry and parameter packing of the vectorised PEPS.

Method section, Eq. (4): the vectorised density matrix is a PEPS on an
L1 x L2 square lattice whose site tensors T_i carry one merged physical index
S_i = (s_i, s'_i) of dimension d^2.  Open boundaries: a virtual leg that
points out of the lattice has dimension 1, every other leg has dimension D.

Conventions (readings; the paper fixes none of them):
  * site (r, c), r = 0..L1-1 top to bottom, c = 0..L2-1 left to right,
    linear index i = r * L2 + c;
  * T_i[S][l][u][r][d] (left, up, right, down), row-major;
  * S = s * d + s'  (ket digit s, bra digit s');
  * theta = concatenation over i of the flattened T_i;
  * one O row = concatenation over i of a [l][u][r][d] block (the slice S_i
    of site i is implied by the configuration).
"""
from __future__ import annotations

import numpy as np

MODEL_HEISENBERG = 0
MODEL_HUBBARD = 1


class Lattice:
    """Shape of one problem: lattice, bond dimensions and model couplings."""

    def __init__(self, L1, L2, D, chi, d=2, model=MODEL_HEISENBERG,
                 J1=1.0, J2=0.0, t=1.0, U=0.0, mu=0.0):
        if L1 < 2 or L2 < 2:
            raise ValueError("lattice must be at least 2 x 2")
        self.L1, self.L2, self.D, self.chi, self.d = int(L1), int(L2), int(D), int(chi), int(d)
        self.d2 = self.d * self.d
        self.N = self.L1 * self.L2
        self.model = int(model)
        self.J1, self.J2 = float(J1), float(J2)
        self.t, self.U, self.mu = float(t), float(U), float(mu)

    # -- geometry ---------------------------------------------------------
    def site(self, r, c):
        return r * self.L2 + c

    def leg_dims(self, r, c):
        """(Dl, Du, Dr, Dd) of site (r, c); boundary legs have dimension 1."""
        D = self.D
        return (1 if c == 0 else D,
                1 if r == 0 else D,
                1 if c == self.L2 - 1 else D,
                1 if r == self.L1 - 1 else D)

    def block_size(self, r, c):
        Dl, Du, Dr, Dd = self.leg_dims(r, c)
        return Dl * Du * Dr * Dd

    # -- packing ----------------------------------------------------------
    def param_offsets(self):
        """Start of each site's d^2 * block in theta, and N_p."""
        off, acc = [], 0
        for r in range(self.L1):
            for c in range(self.L2):
                off.append(acc)
                acc += self.d2 * self.block_size(r, c)
        return off, acc

    def orow_offsets(self):
        """Start of each site's block in one O row, and nnz per row."""
        off, acc = [], 0
        for r in range(self.L1):
            for c in range(self.L2):
                off.append(acc)
                acc += self.block_size(r, c)
        return off, acc

    @property
    def n_params(self):
        return self.param_offsets()[1]

    @property
    def nnz(self):
        return self.orow_offsets()[1]

    def site_tensor(self, theta, r, c):
        """T_{rc} as an array [d2, Dl, Du, Dr, Dd] (a view into theta)."""
        off, _ = self.param_offsets()
        dims = self.leg_dims(r, c)
        n = self.d2 * int(np.prod(dims))
        o = off[self.site(r, c)]
        return theta[o:o + n].reshape((self.d2,) + dims)

    def row_slices(self, theta, config, r):
        """W_c = T_{rc}^{S_rc} for c = 0..L2-1, each [l, u, r, d]."""
        cfg = np.asarray(config).reshape(self.L1, self.L2)
        return [self.site_tensor(theta, r, c)[int(cfg[r, c])] for c in range(self.L2)]

    # -- local basis --------------------------------------------------------
    def ket(self, S):
        return int(S) // self.d

    def bra(self, S):
        return int(S) % self.d

    def merge(self, s, sp):
        return int(s) * self.d + int(sp)

    # -- bonds ------------------------------------------------------------
    def bonds_h(self):
        return [((r, c), (r, c + 1)) for r in range(self.L1) for c in range(self.L2 - 1)]

    def bonds_v(self):
        return [((r, c), (r + 1, c)) for r in range(self.L1 - 1) for c in range(self.L2)]

    def bonds_d(self):
        """Next-nearest-neighbour (diagonal) bonds, both orientations."""
        out = []
        for r in range(self.L1 - 1):
            for c in range(self.L2 - 1):
                out.append(((r, c), (r + 1, c + 1)))
                out.append(((r, c + 1), (r + 1, c)))
        return out

    def n_site_moves(self):
        """Site proposals per site: spin (s,s) -> (s~,s~); Hubbard: one per
        species (toggle n_sigma of ket and bra together)."""
        return 1 if self.model == MODEL_HEISENBERG else 2

    def n_bond_moves(self):
        """Bond proposals per bond: ket and bra exchange (spin); ket and bra
        exchange of each species separately (Hubbard)."""
        return 2 if self.model == MODEL_HEISENBERG else 4

    def n_slots(self):
        """Proposal slots per sweep (every slot owns one uniform)."""
        L1, L2, nb = self.L1, self.L2, self.n_bond_moves()
        return L1 * (nb * (L2 - 1) + self.n_site_moves() * L2) + (L1 - 1) * nb * L2
