"""Independent references that pin the splitting oracle (test infrastructure only).

* Brute force on the full lifted matrix: exp(-i t H) of H = D + V^1 + V^2
  (eq. 3.5) via scipy.linalg.expm (Pade scaling-and-squaring, not eigh), and the
  Lie / Strang products of App. A formed from dense exponentials of the full
  split operators.  Only for small N.
* Commensurate supercell: for L1 = 1 and L2 = p/q (q, p coprime) the lifted
  wavevector 2 pi (m + n q / p) takes the values 2 pi k / p, k = p m + q n, i.e.
  the plane waves of the period-p supercell.  Summing lifted coefficients with
  equal k commutes with D, V^1 and V^2 (V^1 shifts k by multiples of p, V^2 by
  multiples of q), so the projected lifted dynamics must equal the same split
  computed directly in the supercell basis, up to cutoff-truncation effects.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from . import lifted


def full_split_operators(sys, kappa: float = 0.0):
    """Dense kappa D, H_1 = (1-kappa)/2 D + V^1, H_2 = (1-kappa)/2 D + V^2 on the full set."""
    D, V1, V2 = lifted.dense_lifted(sys.A1, sys.A2, sys.mn, sys.pot1, sys.pot2)
    return kappa * D, (1.0 - kappa) / 2.0 * D + V1, (1.0 - kappa) / 2.0 * D + V2


def exact_flow(sys, c: np.ndarray, t: float) -> np.ndarray:
    """exp(-i t H) c on the full lifted matrix (no splitting)."""
    D, V1, V2 = lifted.dense_lifted(sys.A1, sys.A2, sys.mn, sys.pot1, sys.pot2)
    return scipy.linalg.expm(-1j * t * (D + V1 + V2)) @ c


def dense_split_step_matrix(sys, tau: float, scheme: str, kappa: float = 0.0) -> np.ndarray:
    """One Lie or Strang step as a dense N x N matrix built from full-size expm's."""
    Dk, H1, H2 = full_split_operators(sys, kappa)
    E = lambda A, t: scipy.linalg.expm(-1j * t * A)  # noqa: E731
    if scheme == "lie":
        return E(H2, tau) @ E(Dk, tau) @ E(H1, tau)
    return E(H1, tau / 2) @ E(Dk, tau / 2) @ E(H2, tau) @ E(Dk, tau / 2) @ E(H1, tau / 2)


class Supercell:
    """Direct 1D supercell model for L1 = 1, L2 = p/q (commensurate counter-case)."""

    def __init__(self, p: int, q: int, pot1: dict, pot2: dict, kmax: int):
        self.p, self.q = int(p), int(q)
        assert math.gcd(self.p, self.q) == 1
        self.k = np.arange(-kmax, kmax + 1)
        self.M = len(self.k)
        Kvec = 2.0 * math.pi * self.k / self.p
        self.D = np.diag(0.5 * Kvec ** 2).astype(np.complex128)
        self.V1 = np.zeros((self.M, self.M), dtype=np.complex128)
        self.V2 = np.zeros((self.M, self.M), dtype=np.complex128)
        for a in range(self.M):
            for b in range(self.M):
                dk = int(self.k[a] - self.k[b])
                if dk % self.p == 0:
                    self.V1[a, b] = pot1.get((dk // self.p,), 0.0)
                if dk % self.q == 0:
                    self.V2[a, b] = pot2.get((dk // self.q,), 0.0)

    def project(self, mn: np.ndarray, c: np.ndarray) -> np.ndarray:
        """(Pi c)_k = sum over lifted (m, n) with p m + q n = k."""
        kk = self.p * mn[:, 0] + self.q * mn[:, 1]
        out = np.zeros((self.M,) + c.shape[1:], dtype=np.complex128)
        np.add.at(out, kk - self.k[0], c)
        return out

    def strang_step_matrix(self, tau: float, kappa: float = 0.0) -> np.ndarray:
        H1 = (1.0 - kappa) / 2.0 * self.D + self.V1
        H2 = (1.0 - kappa) / 2.0 * self.D + self.V2
        E = lambda A, t: scipy.linalg.expm(-1j * t * A)  # noqa: E731
        return (E(H1, tau / 2) @ E(kappa * self.D, tau / 2) @ E(H2, tau)
                @ E(kappa * self.D, tau / 2) @ E(H1, tau / 2))

    def lie_step_matrix(self, tau: float, kappa: float = 0.0) -> np.ndarray:
        H1 = (1.0 - kappa) / 2.0 * self.D + self.V1
        H2 = (1.0 - kappa) / 2.0 * self.D + self.V2
        E = lambda A, t: scipy.linalg.expm(-1j * t * A)  # noqa: E731
        return E(H2, tau) @ E(kappa * self.D, tau) @ E(H1, tau)


def dense_rational_step_matrix(sys, tau: float, scheme: str, kappa: float = 0.0) -> np.ndarray:
    """One Lie-BE (Alg. 2) or Strang-CN (eq. 4.6) step as a dense N x N matrix, from linear
    solves with the full split operators (kinetic share by its exact exponential)."""
    Dk, H1, H2 = full_split_operators(sys, kappa)
    N = H1.shape[0]
    I = np.eye(N)
    E = lambda A, t: scipy.linalg.expm(-1j * t * A)  # noqa: E731
    if scheme == "lie_be":
        B = lambda A, t: np.linalg.solve(I + 1j * t * A, I)  # noqa: E731
        return B(H2, tau) @ E(Dk, tau) @ B(H1, tau)
    C = lambda A, t: np.linalg.solve(I + 0.5j * t * A, I - 0.5j * t * A)  # noqa: E731
    return C(H1, tau / 2) @ E(Dk, tau / 2) @ C(H2, tau) @ E(Dk, tau / 2) @ C(H1, tau / 2)
