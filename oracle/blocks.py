"""Lifted systems whose layers share index blocks (oracle; test infrastructure only).

Example 3 of Sec. 5 is a two-dimensional system that is periodic in y and incommensurate in
x.  It is lifted with three indices: m and n for the two incommensurate periods in x, and p
for the shared period in y, so a plane wave is exp(i (G_1 m + G_2 n) x + i G_3 p y).  Each
potential term is a product of an x-factor of one layer and a y-factor, so V^1 couples the
pair (m, p) and V^2 couples (n, p).

General form built here:
  * index blocks b = 0 .. B-1, block b an integer vector m_b in Z^{d_b}, with a physical
    embedding R_b (D x d_b): the wavevector is K = sum_b R_b m_b, D = diag(|K|^2 / 2);
  * cutoff groups: every group g keeps sum_{b in g} |R_b m_b|^2 <= 2 Ec (relative tolerance
    1e-12, as for the two-layer set), and the set is the product over groups;
  * layers j = 1 .. L, layer j coupling the contiguous block range [s_j, e_j):
        V^j_{(m), (m')} = v^(j)_{(m_b - m'_b), b in [s_j, e_j)}  if m_b = m'_b for b outside;
  * H = kappa D + sum_j H_j,  H_j = (1 - kappa)/L D + V^j.
A layer-j fibre fixes every block outside [s_j, e_j).  Canonical order is lexicographic in
(m_0, ..., m_{B-1}); fibres are ordered by their fixed blocks (lexicographic, block order),
rows ascending.  One block per layer with a single group is the L-layer ball set of
`multilayer`; one group per block is its product set.  The compositions are those of
`multilayer.MultiSplitPlan`, which works on any system with this interface.
"""
from __future__ import annotations

import itertools

import numpy as np


def block_candidates(R: np.ndarray, lim: float):
    """All m in Z^{d_b} with |R m|^2 <= lim, lexicographic, with |R m|^2.  The bound
    |m_k| <= |row_k(R^+)| |R m| (R^+ the pseudo-inverse, R of full column rank) covers them."""
    R = np.asarray(R, dtype=np.float64)
    Rp = np.linalg.pinv(R)
    bnd = [int(np.floor(np.sqrt(lim) * np.linalg.norm(Rp[k]))) + 1 for k in range(R.shape[1])]
    out = []
    for m in itertools.product(*[range(-b, b + 1) for b in bnd]):
        g = R @ np.array(m, dtype=np.float64)
        s = float(g @ g)
        if s <= lim:
            out.append((m, s))
    return out


class BlockSystem:
    """Index set, wavevectors, fibres and fibre Hamiltonians of a block-lifted system."""

    def __init__(self, Rs, groups, Ec: float, layers, pots):
        self.Rs = [np.asarray(R, dtype=np.float64) for R in Rs]
        self.D = self.Rs[0].shape[0]
        self.dims = [R.shape[1] for R in self.Rs]
        self.off = np.concatenate([[0], np.cumsum(self.dims)]).astype(int)
        self.groups = [list(g) for g in groups]
        self.layers = [tuple(x) for x in layers]
        self.L = len(self.layers)
        self.Ec = float(Ec)
        self.pots = [{tuple(int(x) for x in k): complex(v) for k, v in p.items()} for p in pots]
        lim = 2.0 * self.Ec * (1.0 + 1e-12)
        cands = [block_candidates(R, lim) for R in self.Rs]
        group_of = {b: g for g, blocks in enumerate(self.groups) for b in blocks}
        rows = []
        for combo in itertools.product(*cands):
            sums = [0.0] * len(self.groups)
            for b, (_, s) in enumerate(combo):
                sums[group_of[b]] += s
            if all(x <= lim for x in sums):
                rows.append([x for m, _ in combo for x in m])
        self.mn = np.array(rows, dtype=np.int64).reshape(-1, int(self.off[-1]))
        self.N = self.mn.shape[0]
        K = np.zeros((self.N, self.D))
        for b, R in enumerate(self.Rs):
            K += self.mn[:, self.off[b]:self.off[b + 1]] @ R.T
        self.K = K
        self.K2 = (K * K).sum(axis=1)
        self.fib = {j + 1: self._fibres(j) for j in range(self.L)}

    def coupled(self, j: int):
        """Columns of the lifted index that V^(j+1) couples."""
        s, e = self.layers[j]
        return list(range(self.off[s], self.off[e]))

    def _fibres(self, j: int):
        cols = set(self.coupled(j))
        keep = [k for k in range(self.mn.shape[1]) if k not in cols]
        groups: dict = {}
        for i in range(self.N):
            groups.setdefault(tuple(int(x) for x in self.mn[i, keep]), []).append(i)
        return [(k, np.array(groups[k], dtype=np.int64)) for k in sorted(groups)]

    def fibre_hamiltonian(self, layer: int, rows: np.ndarray, kappa: float) -> np.ndarray:
        """H_j on one fibre: (1 - kappa)/L D + V^j restricted to the fibre."""
        cols = self.coupled(layer - 1)
        own = self.mn[rows][:, cols]
        diff = own[:, None, :] - own[None, :, :]
        H = np.zeros((len(rows), len(rows)), dtype=np.complex128)
        for p, v in self.pots[layer - 1].items():
            H[np.all(diff == np.array(p)[None, None, :], axis=2)] += v
        H[np.arange(len(rows)), np.arange(len(rows))] += (1.0 - kappa) / self.L * 0.5 * self.K2[rows]
        return H

    def dense(self, kappa: float = 0.0):
        """Dense kappa D and H_1 .. H_L on the whole set, V^j entry by entry."""
        lookup = {tuple(int(x) for x in row): i for i, row in enumerate(self.mn)}
        D = np.diag(0.5 * self.K2).astype(np.complex128)
        Hs = []
        for j in range(self.L):
            cols = self.coupled(j)
            V = np.zeros((self.N, self.N), dtype=np.complex128)
            for i, row in enumerate(self.mn):
                for p, v in self.pots[j].items():
                    src = row.copy()
                    src[cols] -= np.array(p)
                    k = lookup.get(tuple(int(x) for x in src))
                    if k is not None:
                        V[i, k] += v
            Hs.append((1.0 - kappa) / self.L * D + V)
        return kappa * D, Hs


def example3(Ec: float, s1: float = 1.0, s2: float = 2.0, beta: float = (5.0 ** 0.5 - 1.0) / 2.0):
    """Example 3: V = s1 cos^2(beta x) cos^2(pi y / 2) + s2 cos^2(x) cos^2(pi y / 2).
    cos^2(a z) = 1/2 + (e^{2iaz} + e^{-2iaz})/4, so the x-factors have reciprocal vectors
    G_1 = 2 beta and G_2 = 2, the y-factor G_3 = pi, and each layer's coefficients over its
    (x, y) block pair are s_j a_k a_l with a_0 = 1/2, a_{+-1} = 1/4.  Blocks in the order
    (m, p, n) make layer 1 couple blocks [0, 2) and layer 2 blocks [1, 3); the cutoff groups
    are (m, n) (the lifted x-set) and p."""
    a = {0: 0.5, 1: 0.25, -1: 0.25}
    pot = lambda s: {(k, l): s * a[k] * a[l] for k in a for l in a}  # noqa: E731
    pot2 = {(l, k): v for (k, l), v in pot(s2).items()}  # layer 2 couples (p, n)
    Rs = [np.array([[2.0 * beta], [0.0]]), np.array([[0.0], [np.pi]]), np.array([[2.0], [0.0]])]
    return BlockSystem(Rs, [[0, 2], [1]], Ec, [(0, 2), (1, 3)], [pot(s1), pot2])
