"""Observables on lifted coefficients (oracle; test infrastructure only).

Mass (eq. 2.3): by the averaged orthonormality of the lifted plane waves
(eq. 3.1), N(psi) = sum_{(m,n) in I} |phi_mn|^2 (as used in the proof of Thm 4.4).
Energy (eq. 2.4): the averaged kinetic term gives 1/2 |K|^2 |phi|^2 per mode and
the averaged potential terms give phi^H V^j phi, so E = phi^H (D + V^1 + V^2) phi.
Fibre mass: sum of |phi|^2 over the rows of one fibre (a partial mass).
"""
from __future__ import annotations

import numpy as np


def mass(c: np.ndarray) -> np.ndarray:
    """Per-wavepacket mass sum_i |c_iw|^2."""
    c = c.reshape(c.shape[0], -1)
    return (c.real ** 2 + c.imag ** 2).sum(axis=0)


def energy(sys, c: np.ndarray) -> np.ndarray:
    """Per-wavepacket energy Re c^H (D + V^1 + V^2) c, with V^j applied entry by entry.

    (V^1 c)_{(m,n)} = sum_p v1_p c_{(m-p, n)} over pairs inside I (eq. 3.3).
    """
    c = c.reshape(c.shape[0], -1)
    d = sys.d
    lookup = {tuple(int(x) for x in row): i for i, row in enumerate(sys.mn)}
    Hc = 0.5 * sys.K2[:, None] * c
    for i, row in enumerate(sys.mn):
        m, n = row[:d], row[d:]
        for p, v in sys.pot1.items():
            j = lookup.get(tuple(int(x) for x in np.concatenate([m - np.array(p), n])))
            if j is not None:
                Hc[i] += v * c[j]
        for q, v in sys.pot2.items():
            j = lookup.get(tuple(int(x) for x in np.concatenate([m, n - np.array(q)])))
            if j is not None:
                Hc[i] += v * c[j]
    return np.real((c.conj() * Hc).sum(axis=0))


def fibre_mass(sys, c: np.ndarray, layer: int) -> np.ndarray:
    """[nfibres, W] partial masses over the fibres of ``layer``."""
    c = c.reshape(c.shape[0], -1)
    out = np.zeros((len(sys.fib[layer]), c.shape[1]))
    for f, (_, rows) in enumerate(sys.fib[layer]):
        out[f] = (np.abs(c[rows]) ** 2).sum(axis=0)
    return out
