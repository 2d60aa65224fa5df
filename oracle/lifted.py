"""Lifted plane-wave discretisation (oracle; test infrastructure only).

Sec. 2: lattices R_j = A_j Z^d, reciprocal lattices 2 pi A_j^{-T} Z^d.
Sec. 3: plane waves e^{i(G1m + G2n).x} indexed by (m, n) in a cutoff set I;
eq. (3.6): D diagonal with 1/2 |G1m + G2n|^2, V^1 couples (m,n) to (m',n)
through v^(1)_{m-m'}, V^2 couples (m,n) to (m,n') through v^(2)_{n-n'}.

Index-set reading.  The paper's set is the product I1 x I2 with
|G1m|^2 <= 2Ec and |G2n|^2 <= 2Ec.  The workloads use the ball
|G1m|^2 + |G2n|^2 <= 2Ec.  Both are provided; a boundary point is kept when
s <= 2Ec (1 + 1e-12), with s = sum_k (G1m)_k^2 + sum_k (G2n)_k^2.
Canonical order: lexicographic in (m_1..m_d, n_1..n_d).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

TIE = 1.0e-12


def reciprocal(A: np.ndarray) -> np.ndarray:
    """B = 2 pi A^{-T}: columns are the reciprocal primitive vectors (Sec. 2)."""
    return 2.0 * math.pi * np.linalg.inv(np.asarray(A, dtype=np.float64)).T


def _layer_candidates(B: np.ndarray, Ec: float):
    """All m in Z^d with |B m|^2 <= 2Ec (1+TIE), plus their |B m|^2."""
    d = B.shape[0]
    r = math.sqrt(2.0 * Ec * (1.0 + TIE))
    Binv = np.linalg.inv(B)
    # |m_k| = |(B^{-1} G)_k| <= |row_k(B^{-1})| |G|
    bounds = [int(math.floor(r * np.linalg.norm(Binv[k, :]))) + 1 for k in range(d)]
    ranges = [range(-b, b + 1) for b in bounds]
    ms = np.array(list(itertools.product(*ranges)), dtype=np.int64).reshape(-1, d)
    g = ms.astype(np.float64) @ B.T
    s = (g * g).sum(axis=1)
    keep = s <= 2.0 * Ec * (1.0 + TIE)
    return ms[keep], s[keep]


def index_set(A1, A2, Ec: float, cutoff: str = "ball") -> np.ndarray:
    """Lifted index set I as an int64 array [N, 2d] in canonical order (Sec. 3)."""
    B1, B2 = reciprocal(A1), reciprocal(A2)
    d = B1.shape[0]
    m, s1 = _layer_candidates(B1, Ec)
    n, s2 = _layer_candidates(B2, Ec)
    if cutoff == "product":
        keep = np.ones((len(m), len(n)), dtype=bool)
    elif cutoff == "ball":
        keep = (s1[:, None] + s2[None, :]) <= 2.0 * Ec * (1.0 + TIE)
    else:
        raise ValueError(f"unknown cutoff {cutoff!r}")
    im, jn = np.nonzero(keep)
    mn = np.concatenate([m[im], n[jn]], axis=1)
    order = np.lexsort(tuple(mn[:, k] for k in reversed(range(2 * d))))
    return mn[order]


def lifted_wavevectors(A1, A2, mn: np.ndarray) -> np.ndarray:
    """K_i = G1m + G2n for every lifted index (Sec. 3, basis functions)."""
    B1, B2 = reciprocal(A1), reciprocal(A2)
    d = B1.shape[0]
    return mn[:, :d].astype(np.float64) @ B1.T + mn[:, d:].astype(np.float64) @ B2.T


def fibres(mn: np.ndarray, layer: int):
    """Fibres of layer ``layer`` (Sec. 3, block structure of V^1 and permuted V^2).

    Layer 1: for each n, the rows {i : n_i = n} (V^1 couples only these).
    Layer 2: for each m, the rows {i : m_i = m}.
    Returns a list of (key tuple, int64 row array ascending), keys in lexicographic order.
    """
    d = mn.shape[1] // 2
    key = mn[:, d:] if layer == 1 else mn[:, :d]
    groups: dict = {}
    for i in range(mn.shape[0]):
        groups.setdefault(tuple(int(x) for x in key[i]), []).append(i)
    return [(k, np.array(groups[k], dtype=np.int64)) for k in sorted(groups)]


def dense_lifted(A1, A2, mn: np.ndarray, pot1: dict, pot2: dict):
    """Dense D, V^1, V^2 of eq. (3.6) restricted to I (only for small N).

    D_{i,i} = 1/2 |K_i|^2;  V^1_{i,i'} = v1_{m_i - m_i'} if n_i = n_i';
    V^2_{i,i'} = v2_{n_i - n_i'} if m_i = m_i'.
    """
    N = mn.shape[0]
    d = mn.shape[1] // 2
    K = lifted_wavevectors(A1, A2, mn)
    D = np.diag(0.5 * (K * K).sum(axis=1)).astype(np.complex128)
    V1 = np.zeros((N, N), dtype=np.complex128)
    V2 = np.zeros((N, N), dtype=np.complex128)
    for i in range(N):
        mi, ni = tuple(mn[i, :d]), tuple(mn[i, d:])
        for ip in range(N):
            mj, nj = tuple(mn[ip, :d]), tuple(mn[ip, d:])
            if ni == nj:
                diff = tuple(a - b for a, b in zip(mi, mj))
                V1[i, ip] = pot1.get(diff, 0.0)
            if mi == mj:
                diff = tuple(a - b for a, b in zip(ni, nj))
                V2[i, ip] = pot2.get(diff, 0.0)
    return D, V1, V2
