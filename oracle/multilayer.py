"""Layer splitting for systems of L >= 2 layers (oracle; test infrastructure only).

The method carries over directly to more than two layers (Sec. 2, Sec. 3, Sec. 4 opening,
Sec. 6): with L periodic layers of lattices A_j and potentials v^(j), the plane waves are lifted
to indices (m_1, ..., m_L) in Z^{dL} with wavevector K = G_1 m_1 + ... + G_L m_L, the kinetic
part is D = diag(|K|^2 / 2), and V^j couples only m_j (eq. 3.6 layer by layer):
    V^j_{(m), (m')} = v^(j)_{m_j - m'_j} if m_i = m'_i for all i != j.
A layer-j fibre fixes every index but m_j (the block structure of Sec. 3 for each layer).

Kinetic share kappa: H = kappa D + sum_j H_j, H_j = (1 - kappa)/L D + V^j.
Compositions (App. A, generalised to L parts):
    Lie    : F_1(tau), ..., F_{L-1}(tau), Phase(kappa tau), F_L(tau)
    Strang : F_1(tau/2), ..., F_{L-1}(tau/2), Phase(kappa tau/2), F_L(tau), Phase(kappa tau/2),
             F_{L-1}(tau/2), ..., F_1(tau/2)
    Yoshida: S(g1 tau) S(g0 tau) S(g1 tau) with S the Strang step, g1 = 1 / (2 - 2^(1/3)),
             g0 = 1 - 2 g1 (fourth order; App. A points to such higher-order compositions)
For L = 2 these are the two-layer schemes of `splitting`.  Canonical order of the index set is
lexicographic in (m_1, ..., m_L); fibres of layer j are ordered lexicographically by their fixed
indices (in layer order) and list their rows in canonical order.
"""
from __future__ import annotations

import itertools

import numpy as np


def reciprocal(A: np.ndarray) -> np.ndarray:
    """G = 2 pi A^{-T}: G m is the reciprocal vector of integer index m (Sec. 2)."""
    return 2.0 * np.pi * np.linalg.inv(np.asarray(A, dtype=np.float64)).T


def index_set(As, Ec: float, cutoff: str = "ball") -> np.ndarray:
    """All (m_1, ..., m_L) with sum_j |G_j m_j|^2 <= 2 Ec (ball, with the relative tolerance
    1e-12 of the two-layer set) or |G_j m_j|^2 <= 2 Ec for every j (product), in lexicographic
    order; shape [N, L d]."""
    lim = 2.0 * Ec * (1.0 + 1e-12)
    cands = []
    for A in As:
        A = np.asarray(A, dtype=np.float64)
        d = A.shape[0]
        G = reciprocal(A)
        # |m_k| <= |row_k(G^{-1})| |G m| bounds every component
        Ginv = np.linalg.inv(G)
        bnd = [int(np.floor(np.sqrt(lim) * np.linalg.norm(Ginv[k]))) + 1 for k in range(d)]
        layer = []
        for m in itertools.product(*[range(-b, b + 1) for b in bnd]):
            g = G @ np.array(m, dtype=np.float64)
            s = float(g @ g)
            if s <= lim:
                layer.append((m, s))
        cands.append(layer)
    rows = []
    for combo in itertools.product(*cands):
        s = sum(c[1] for c in combo)
        if cutoff == "ball" and not s <= lim:
            continue
        rows.append([x for c in combo for x in c[0]])
    d = np.asarray(As[0]).shape[0]
    return np.array(rows, dtype=np.int64).reshape(-1, len(As) * d)


def fibres(mn: np.ndarray, layer: int, L: int, d: int):
    """Fibres of `layer` (1-based): groups of rows with equal indices outside block `layer`,
    keys in lexicographic order, rows ascending."""
    keep = [k for k in range(L * d) if not (layer - 1) * d <= k < layer * d]
    groups: dict = {}
    for i in range(mn.shape[0]):
        groups.setdefault(tuple(int(x) for x in mn[i, keep]), []).append(i)
    return [(k, np.array(groups[k], dtype=np.int64)) for k in sorted(groups)]


class MultiLifted:
    """An L-layer lifted system: index set, wavevectors, fibres and potentials."""

    def __init__(self, d: int, As, Ec: float, cutoff: str, pots):
        self.d = int(d)
        self.L = len(As)
        self.As = [np.asarray(A, dtype=np.float64).reshape(d, d) for A in As]
        self.Gs = [reciprocal(A) for A in self.As]
        self.Ec = float(Ec)
        self.pots = [{tuple(int(x) for x in k): complex(v) for k, v in p.items()} for p in pots]
        self.mn = index_set(self.As, Ec, cutoff)
        self.N = self.mn.shape[0]
        K = np.zeros((self.N, d))
        for j in range(self.L):
            K += self.mn[:, j * d:(j + 1) * d] @ self.Gs[j].T
        self.K = K
        self.K2 = (K * K).sum(axis=1)
        self.fib = {j: fibres(self.mn, j, self.L, d) for j in range(1, self.L + 1)}

    def fibre_hamiltonian(self, layer: int, rows: np.ndarray, kappa: float) -> np.ndarray:
        """H_j on one fibre: (1 - kappa)/L * D + V^j restricted to the fibre."""
        d = self.d
        own = self.mn[rows][:, (layer - 1) * d:layer * d]
        diff = own[:, None, :] - own[None, :, :]
        H = np.zeros((len(rows), len(rows)), dtype=np.complex128)
        for p, v in self.pots[layer - 1].items():
            H[np.all(diff == np.array(p)[None, None, :], axis=2)] += v
        H[np.arange(len(rows)), np.arange(len(rows))] += (1.0 - kappa) / self.L * 0.5 * self.K2[rows]
        return H

    def dense(self, kappa: float = 0.0):
        """Dense kappa D and H_1..H_L on the whole set (entrywise V^j as in the module docstring)."""
        d, L = self.d, self.L
        lookup = {tuple(int(x) for x in row): i for i, row in enumerate(self.mn)}
        D = np.diag(0.5 * self.K2).astype(np.complex128)
        Hs = []
        for j in range(L):
            V = np.zeros((self.N, self.N), dtype=np.complex128)
            for i, row in enumerate(self.mn):
                for p, v in self.pots[j].items():
                    src = row.copy()
                    src[j * d:(j + 1) * d] -= np.array(p)
                    k = lookup.get(tuple(int(x) for x in src))
                    if k is not None:
                        V[i, k] += v
            Hs.append((1.0 - kappa) / L * D + V)
        return kappa * D, Hs


class MultiSplitPlan:
    """Fibre sub-steps of every layer, cached per (layer, t); unmerged compositions.

    ``flow`` selects the sub-step: ``"exact"`` exp(-i t H_j) (eigh), ``"be"`` the backward-Euler
    solve (I + i t H_j)^{-1} (Alg. 2, eqs. 4.3-4.4), or ``"cn"`` the Crank-Nicolson solve
    (I + i t H_j / 2)^{-1}(I - i t H_j / 2) (eq. 4.6), formed by linear solves with the fibre
    matrix.  The rational flows are used with the Lie (BE) and Strang (CN) compositions, as
    for two layers."""

    def __init__(self, sys: MultiLifted, kappa: float = 0.0, flow: str = "exact"):
        self.sys = sys
        self.kappa = float(kappa)
        self.flow = flow
        self._eig = {}
        self._P = {}

    def propagators(self, layer: int, t: float):
        key = (layer, float(t))
        if key in self._P:
            return self._P[key]
        if self.flow == "exact":
            if layer not in self._eig:
                self._eig[layer] = [np.linalg.eigh(self.sys.fibre_hamiltonian(layer, rows, self.kappa))
                                    for _, rows in self.sys.fib[layer]]
            self._P[key] = [(U * np.exp(-1j * t * lam)[None, :]) @ U.conj().T for lam, U in self._eig[layer]]
        else:
            out = []
            for _, rows in self.sys.fib[layer]:
                H = self.sys.fibre_hamiltonian(layer, rows, self.kappa)
                I = np.eye(len(rows))
                if self.flow == "be":
                    out.append(np.linalg.solve(I + 1j * t * H, I))
                else:
                    out.append(np.linalg.solve(I + 0.5j * t * H, I - 0.5j * t * H))
            self._P[key] = out
        return self._P[key]

    def apply_fibres(self, c, layer: int, t: float):
        c = np.asarray(c, dtype=np.complex128)
        out = c.copy()
        for (_, rows), P in zip(self.sys.fib[layer], self.propagators(layer, t)):
            out[rows] = P @ c[rows]
        return out

    def apply_phase(self, c, t: float):
        ph = np.exp(-1j * self.kappa * t * 0.5 * self.sys.K2)
        return c * (ph[:, None] if c.ndim == 2 else ph)

    def lie_step(self, c, tau: float):
        L = self.sys.L
        for j in range(1, L):
            c = self.apply_fibres(c, j, tau)
        if self.kappa != 0.0:
            c = self.apply_phase(c, tau)
        return self.apply_fibres(c, L, tau)

    def strang_step(self, c, tau: float):
        L = self.sys.L
        for j in range(1, L):
            c = self.apply_fibres(c, j, tau / 2)
        if self.kappa != 0.0:
            c = self.apply_phase(c, tau / 2)
        c = self.apply_fibres(c, L, tau)
        if self.kappa != 0.0:
            c = self.apply_phase(c, tau / 2)
        for j in range(L - 1, 0, -1):
            c = self.apply_fibres(c, j, tau / 2)
        return c

    def yoshida4_step(self, c, tau: float):
        """Symmetric triple jump of Strang steps, applied unmerged: 2 g1 + g0 = 1 and
        2 g1^3 + g0^3 = 0 cancel the third-order error of the composition."""
        g1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
        g0 = 1.0 - 2.0 * g1
        for g in (g1, g0, g1):
            c = self.strang_step(c, g * tau)
        return c

    def evolve(self, c, tau: float, nsteps: int, scheme: str = "strang"):
        step = {"strang": self.strang_step, "lie": self.lie_step, "yoshida4": self.yoshida4_step}[scheme]
        for _ in range(nsteps):
            c = step(c, tau)
        return c
