"""Pins of the block-lifted oracle (layers that share index blocks, Example 3): exact reduction to
the L-layer oracle, dense brute force, a commensurate Example 3 against the same split computed
directly in the physical plane-wave basis of its supercell, orders 1 and 2, unitarity and the
free particle."""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import blocks
from oracle import multilayer as ml
from paper_2103_14897_amd import workloads as wl


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("spec", [wl.chain_layers(120.0), wl.chain_layers(100.0, cutoff="product"),
                                  wl.twisted_layers(40.0, thetas_deg=(-2.0, 2.0), v=(1.0, 0.5))],
                         ids=["chain3", "chain3_product", "twisted2"])
def test_one_block_per_layer_reduces_to_the_layer_oracle(spec):
    O = ml.MultiLifted(spec.d, spec.As, spec.Ec, spec.cutoff, spec.pots)
    L = spec.L
    groups = [list(range(L))] if spec.cutoff == "ball" else [[b] for b in range(L)]
    B = blocks.BlockSystem([ml.reciprocal(A) for A in spec.As], groups, spec.Ec,
                           [(j, j + 1) for j in range(L)], spec.pots)
    assert np.array_equal(B.mn, O.mn)
    for j in range(1, L + 1):
        assert [k for k, _ in B.fib[j]] == [k for k, _ in O.fib[j]]
        assert all(np.array_equal(a, b) for (_, a), (_, b) in zip(B.fib[j], O.fib[j]))
    c = wl.random_state(O.N, 2, seed=1)
    for kappa in (0.0, 0.5):
        pb, po = ml.MultiSplitPlan(B, kappa), ml.MultiSplitPlan(O, kappa)
        for scheme in ("lie", "strang", "yoshida4"):
            assert rel(pb.evolve(c, 0.02, 2, scheme), po.evolve(c, 0.02, 2, scheme)) < 1e-13


def example3_small():
    O = blocks.example3(40.0)
    assert 100 < O.N < 600, O.N
    return O


@pytest.mark.parametrize("kappa", [0.0, 1.0])
def test_example3_step_equals_dense_products(kappa):
    O = example3_small()
    plan = ml.MultiSplitPlan(O, kappa)
    Dk, (H1, H2) = O.dense(kappa)
    E = lambda A, t: scipy.linalg.expm(-1j * t * A)  # noqa: E731
    c = wl.random_state(O.N, 2, seed=2)
    tau = 0.04
    assert rel(plan.lie_step(c, tau), E(H2, tau) @ E(Dk, tau) @ E(H1, tau) @ c) < 1e-13
    strang = E(H1, tau / 2) @ E(Dk, tau / 2) @ E(H2, tau) @ E(Dk, tau / 2) @ E(H1, tau / 2)
    assert rel(plan.strang_step(c, tau), strang @ c) < 1e-13


def test_example3_commensurate_supercell():
    """beta = 1/2: the x-wavevector 2 beta m + 2 n = m + 2 n is an integer and the y-wavevector is
    pi p, so the physical system is periodic with period 2 pi in x and 2 in y.  Summing the
    lifted coefficients of equal (m + 2n, p) commutes with D, V^1 (shifts m and p) and V^2
    (shifts n and p), so the projected lifted Strang step equals the same split written directly
    in the physical plane-wave basis (kx, ky) = (a, pi c) (decaying data makes the two
    truncations agree)."""
    s1, s2 = 1.0, 2.0
    O = blocks.example3(200.0, s1=s1, s2=s2, beta=0.5)
    a_idx = O.mn[:, 0] + 2 * O.mn[:, 2]
    c_idx = O.mn[:, 1]
    A, C = int(np.abs(a_idx).max()), int(np.abs(c_idx).max())
    grid = [(a, c) for a in range(-A, A + 1) for c in range(-C, C + 1)]
    pos = {g: i for i, g in enumerate(grid)}
    M = len(grid)
    coef = {0: 0.5, 1: 0.25, -1: 0.25}
    Dp = np.diag([0.5 * (a * a + (np.pi * c) ** 2) for a, c in grid]).astype(np.complex128)
    V1 = np.zeros((M, M), dtype=np.complex128)
    V2 = np.zeros((M, M), dtype=np.complex128)
    for (a, c), i in pos.items():
        for k, ak in coef.items():
            for l, al in coef.items():
                src1 = pos.get((a - k, c - l))      # cos^2(x/2): x-shift 1 per step of m
                if src1 is not None:
                    V1[i, src1] += s1 * ak * al
                src2 = pos.get((a - 2 * k, c - l))  # cos^2(x): x-shift 2 per step of n
                if src2 is not None:
                    V2[i, src2] += s2 * ak * al
    kappa, tau, nsteps = 0.0, 0.01, 15
    E = lambda X, t: scipy.linalg.expm(-1j * t * X)  # noqa: E731
    H1 = (1.0 - kappa) / 2 * Dp + V1
    H2 = (1.0 - kappa) / 2 * Dp + V2
    S = E(H1, tau / 2) @ E(H2, tau) @ E(H1, tau / 2)
    # data decaying in every lifted index
    own = (2 * 0.5 * O.mn[:, 0]) ** 2 + (np.pi * O.mn[:, 1]) ** 2 + (2 * O.mn[:, 2]) ** 2
    c0 = np.exp(-0.5 * (O.K[:, 0] - 1.0) ** 2 - 0.5 * O.K[:, 1] ** 2 - 0.08 * own).astype(np.complex128)
    c0 /= np.linalg.norm(c0)

    def project(x):
        out = np.zeros(M, dtype=np.complex128)
        for i in range(O.N):
            out[pos[(int(a_idx[i]), int(c_idx[i]))]] += x[i]
        return out

    x = ml.MultiSplitPlan(O, kappa).evolve(c0, tau, nsteps, "strang")
    ref = np.linalg.matrix_power(S, nsteps) @ project(c0)
    assert rel(project(x), ref) < 1e-9


@pytest.mark.parametrize("scheme,order", [("lie", 1.0), ("strang", 2.0)])
def test_example3_orders(scheme, order):
    O = example3_small()
    Dk, Hs = O.dense(0.0)
    H = Dk + sum(Hs)
    c0 = wl.random_state(O.N, 1, seed=3)[:, 0]
    T = 0.5
    exact = scipy.linalg.expm(-1j * T * H) @ c0
    plan = ml.MultiSplitPlan(O, 0.0)
    errs = [np.linalg.norm(plan.evolve(c0, T / K, K, scheme) - exact) for K in (80, 160, 320)]
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(s - order) < 0.15 for s in slopes), (errs, slopes)


def test_example3_fibres_unitarity_and_free_particle():
    O = example3_small()
    # layer-1 fibres fix n (the last block), layer-2 fibres fix m (the first block): the
    # latter are contiguous runs of the canonical order
    assert all(len(set(O.mn[r, 2])) == 1 for _, r in O.fib[1])
    assert np.array_equal(np.concatenate([r for _, r in O.fib[2]]), np.arange(O.N))
    c0 = wl.random_state(O.N, 2, seed=4)
    for kappa in (0.0, 0.4):
        c = ml.MultiSplitPlan(O, kappa).evolve(c0, 0.02, 20)
        assert np.abs(np.linalg.norm(c, axis=0) - np.linalg.norm(c0, axis=0)).max() < 1e-12
    free = blocks.example3(40.0, s1=0.0, s2=0.0)
    c = ml.MultiSplitPlan(free, 0.3).evolve(c0, 0.02, 10)
    assert rel(c, c0 * np.exp(-1j * 0.2 * 0.5 * free.K2)[:, None]) < 1e-13
