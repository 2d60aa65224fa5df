"""Exact-flow layer splitting on the lifted coefficient array (oracle; test infrastructure only).

Splitting of H = D + V^1 + V^2 (eq. 3.5).  The paper splits
H = (D/2 + V^1) + (D/2 + V^2) (Sec. 4.2); each part is block diagonal over the
fibres of one layer (Sec. 3), so its exact flow exp(-i t H_j) is one small
dense exponential per fibre.  The layer-splitting theory treats these exact
sub-flows as the semi-discrete limit of Alg. 2 / eq. (4.6) (App. A, App. B).

Kinetic-share reading (kappa).  With 0 <= kappa <= 1,
    H = kappa D + H_1 + H_2,  H_j = (1 - kappa)/2 D + V^j.
kappa = 0 is the paper's split; kappa = 1 puts all of D into an elementwise
phase exp(-i kappa t |K|^2 / 2) (the kinetic sub-step of Alg. 3) and leaves
potential-only fibre Hamiltonians.  Compositions (App. A), applied left to right
in time:
    Lie    : F1(tau), Phase(kappa tau), F2(tau)
    Strang : F1(tau/2), Phase(kappa tau/2), F2(tau), Phase(kappa tau/2), F1(tau/2)
The oracle applies every step unmerged.

Fibre propagator: P(t) = U diag(exp(-i t lambda)) U^H from numpy.linalg.eigh of
the fibre Hamiltonian.
"""
from __future__ import annotations

import numpy as np

from . import lifted


class Lifted:
    """A lifted system: index set, wavevectors, fibres and potentials (Secs. 2-3)."""

    def __init__(self, d, A1, A2, Ec, cutoff, pot1, pot2, mn=None):
        self.d = int(d)
        self.A1 = np.asarray(A1, dtype=np.float64).reshape(d, d)
        self.A2 = np.asarray(A2, dtype=np.float64).reshape(d, d)
        self.Ec = float(Ec)
        self.cutoff = cutoff
        self.pot1 = {tuple(int(x) for x in k): complex(v) for k, v in pot1.items()}
        self.pot2 = {tuple(int(x) for x in k): complex(v) for k, v in pot2.items()}
        self.mn = lifted.index_set(self.A1, self.A2, self.Ec, cutoff) if mn is None else np.asarray(mn)
        self.N = self.mn.shape[0]
        self.K = lifted.lifted_wavevectors(self.A1, self.A2, self.mn)
        self.K2 = (self.K * self.K).sum(axis=1)  # |G1m + G2n|^2
        self.fib = {1: lifted.fibres(self.mn, 1), 2: lifted.fibres(self.mn, 2)}

    @classmethod
    def from_spec(cls, spec):
        return cls(spec.d, spec.A1, spec.A2, spec.Ec, spec.cutoff, spec.pot1, spec.pot2)

    def fibre_hamiltonian(self, layer: int, rows: np.ndarray, kappa: float) -> np.ndarray:
        """H_j restricted to one fibre: (1-kappa)/2 * D + V^j (eqs. 3.6, Sec. 4.2).

        Layer 1 (fixed n): entries v1_{m_a - m_b};  layer 2 (fixed m): v2_{n_a - n_b}.
        """
        d = self.d
        sub = self.mn[rows]
        own = sub[:, :d] if layer == 1 else sub[:, d:]
        pot = self.pot1 if layer == 1 else self.pot2
        L = len(rows)
        H = np.zeros((L, L), dtype=np.complex128)
        diff = own[:, None, :] - own[None, :, :]  # [L, L, d]: m_a - m_b
        for p, v in pot.items():
            H[np.all(diff == np.array(p)[None, None, :], axis=2)] += v
        H[np.arange(L), np.arange(L)] += (1.0 - kappa) / 2.0 * 0.5 * self.K2[rows]
        return H


def propagator_from_hamiltonian(H: np.ndarray, t: float) -> np.ndarray:
    """exp(-i t H) = U diag(exp(-i t lambda)) U^H for Hermitian H (eigh)."""
    lam, U = np.linalg.eigh(H)
    return (U * np.exp(-1j * t * lam)[None, :]) @ U.conj().T


class SplitPlan:
    """Per-fibre propagators for one (system, kappa), cached per (layer, t).

    ``flow`` selects the fibre sub-step: ``"exact"`` exp(-i t H_j) (eigh), ``"be"`` the
    backward-Euler solve (I + i t H_j)^{-1} of Alg. 2 / eqs. (4.3)-(4.4), or ``"cn"`` the
    Crank-Nicolson solve (I + i t H_j / 2)^{-1}(I - i t H_j / 2) of eq. (4.6) (for t = tau/2
    this is (4I + i tau H)^{-1}(4I - i tau H)).  The rational sub-steps are formed by
    linear solves with the fibre matrix, not from its eigenvalues.
    """

    def __init__(self, sys: Lifted, kappa: float = 0.0, flow: str = "exact"):
        self.sys = sys
        self.kappa = float(kappa)
        self.flow = flow
        self._eig = {}
        self._P = {}

    def eig(self, layer: int):
        if layer not in self._eig:
            out = []
            for _, rows in self.sys.fib[layer]:
                H = self.sys.fibre_hamiltonian(layer, rows, self.kappa)
                out.append(np.linalg.eigh(H))
            self._eig[layer] = out
        return self._eig[layer]

    def propagators(self, layer: int, t: float):
        key = (layer, float(t))
        if key not in self._P:
            if self.flow == "exact":
                self._P[key] = [(U * np.exp(-1j * t * lam)[None, :]) @ U.conj().T
                                for lam, U in self.eig(layer)]
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

    def apply_fibres(self, c: np.ndarray, layer: int, t: float) -> np.ndarray:
        """One layer pass: c[rows] <- P_f(t) c[rows] for every fibre f of ``layer``."""
        out = np.array(c, dtype=np.complex128, copy=True)
        for (_, rows), P in zip(self.sys.fib[layer], self.propagators(layer, t)):
            out[rows] = P @ c[rows]
        return out

    def apply_phase(self, c: np.ndarray, t: float) -> np.ndarray:
        """Kinetic phase: c_i <- exp(-i kappa t |K_i|^2 / 2) c_i (Alg. 3 step 1 with share kappa)."""
        ph = np.exp(-1j * self.kappa * t * 0.5 * self.sys.K2)
        return c * (ph[:, None] if c.ndim == 2 else ph)

    def lie_step(self, c: np.ndarray, tau: float) -> np.ndarray:
        c = self.apply_fibres(c, 1, tau)
        if self.kappa != 0.0:
            c = self.apply_phase(c, tau)
        return self.apply_fibres(c, 2, tau)

    def strang_step(self, c: np.ndarray, tau: float) -> np.ndarray:
        c = self.apply_fibres(c, 1, tau / 2)
        if self.kappa != 0.0:
            c = self.apply_phase(c, tau / 2)
        c = self.apply_fibres(c, 2, tau)
        if self.kappa != 0.0:
            c = self.apply_phase(c, tau / 2)
        return self.apply_fibres(c, 1, tau / 2)

    def yoshida4_step(self, c: np.ndarray, tau: float) -> np.ndarray:
        """Fourth-order symmetric composition of three Strang steps (Yoshida's triple jump,
        the higher-order splitting the paper refers to in App. A): S(g1 tau) S(g0 tau) S(g1 tau)
        with g1 = 1 / (2 - 2^(1/3)) and g0 = 1 - 2 g1, so that 2 g1 + g0 = 1 and
        2 g1^3 + g0^3 = 0.  Applied unmerged."""
        g1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
        g0 = 1.0 - 2.0 * g1
        for g in (g1, g0, g1):
            c = self.strang_step(c, g * tau)
        return c

    def evolve(self, c: np.ndarray, tau: float, nsteps: int, scheme: str = "strang",
               callback=None) -> np.ndarray:
        step = {"strang": self.strang_step, "lie": self.lie_step, "yoshida4": self.yoshida4_step}[scheme]
        for k in range(nsteps):
            c = step(c, tau)
            if callback is not None:
                callback(k + 1, c)
        return c
