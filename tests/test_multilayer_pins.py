"""Pins of the L-layer oracle: exact reduction to the two-layer oracle, dense brute force and
splitting orders for three layers, a three-layer commensurate supercell computed directly,
unitarity, reversibility and the free particle."""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import multilayer as ml
from oracle import splitting
from paper_2103_14897_amd import workloads as wl

SQRT2 = math.sqrt(2.0)


def three_chain(Ec, v=(1.0, 0.7, 0.5), L=(1.0, wl.GOLDEN, SQRT2), cutoff="ball"):
    pots = [{(1,): vj, (-1,): vj} for vj in v]
    return ml.MultiLifted(1, [[[x]] for x in L], Ec, cutoff, pots)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("spec", [wl.chain_system(400.0), wl.twisted_system(120.0),
                                  wl.chain_system(300.0, cutoff="product")], ids=["chain", "twisted", "product"])
def test_two_layers_reduce_to_the_two_layer_oracle(spec):
    O2 = splitting.Lifted.from_spec(spec)
    OL = ml.MultiLifted(spec.d, [spec.A1, spec.A2], spec.Ec, spec.cutoff, [spec.pot1, spec.pot2])
    assert np.array_equal(OL.mn, O2.mn)
    for layer in (1, 2):
        assert [k for k, _ in OL.fib[layer]] == [k for k, _ in O2.fib[layer]]
        assert all(np.array_equal(a, b) for (_, a), (_, b) in zip(OL.fib[layer], O2.fib[layer]))
    c = wl.random_state(O2.N, 2, seed=1)
    for kappa in (0.0, 0.5):
        p2, pL = splitting.SplitPlan(O2, kappa), ml.MultiSplitPlan(OL, kappa)
        assert rel(pL.strang_step(c, 0.03), p2.strang_step(c, 0.03)) < 1e-13
        assert rel(pL.lie_step(c, 0.03), p2.lie_step(c, 0.03)) < 1e-13
        assert rel(pL.yoshida4_step(c, 0.03), p2.yoshida4_step(c, 0.03)) < 1e-13


@pytest.mark.parametrize("kappa", [0.0, 1.0])
def test_three_layers_step_equals_dense_products(kappa):
    """Fibre-by-fibre flows equal exponentials of the full lifted H_j (the block structure)."""
    O = three_chain(100.0)
    assert 60 < O.N < 200
    plan = ml.MultiSplitPlan(O, kappa)
    Dk, (H1, H2, H3) = O.dense(kappa)
    E = lambda A, t: scipy.linalg.expm(-1j * t * A)  # noqa: E731
    c = wl.random_state(O.N, 2, seed=2)
    tau = 0.05
    lie = E(H3, tau) @ E(Dk, tau) @ E(H2, tau) @ E(H1, tau)
    strang = (E(H1, tau / 2) @ E(H2, tau / 2) @ E(Dk, tau / 2) @ E(H3, tau) @ E(Dk, tau / 2)
              @ E(H2, tau / 2) @ E(H1, tau / 2))
    assert rel(plan.lie_step(c, tau), lie @ c) < 1e-13
    assert rel(plan.strang_step(c, tau), strang @ c) < 1e-13


@pytest.mark.parametrize("scheme,order,Ks", [("lie", 1.0, (40, 80, 160)), ("strang", 2.0, (40, 80, 160)),
                                             ("yoshida4", 4.0, (80, 160, 320))])
def test_three_layer_orders(scheme, order, Ks):
    O = three_chain(100.0)
    Dk, Hs = O.dense(0.0)
    H = Dk + sum(Hs)
    c0 = wl.random_state(O.N, 1, seed=3)[:, 0]
    T = 0.5
    exact = scipy.linalg.expm(-1j * T * H) @ c0
    plan = ml.MultiSplitPlan(O, 0.0)
    errs = [np.linalg.norm(plan.evolve(c0, T / K, K, scheme) - exact) for K in Ks]
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(s - order) < 0.15 for s in slopes), (errs, slopes)


def test_three_layer_commensurate_supercell():
    """Periods 1, 3/2, 5/4: the lifted wavevector 2 pi (m + 2n/3 + 4l/5) = 2 pi k / 15 with
    k = 15 m + 10 n + 12 l, and V^1, V^2, V^3 shift k by 15, 10, 12.  Summing the lifted
    coefficients of equal k commutes with every part of the split, so the projected lifted
    Strang step equals the same split of the period-15 supercell (decaying data makes the two
    truncations agree)."""
    v = (1.0, 0.7, 0.5)
    O = three_chain(900.0, v=v, L=(1.0, 1.5, 1.25))
    shifts = (15, 10, 12)
    k = 15 * O.mn[:, 0] + 10 * O.mn[:, 1] + 12 * O.mn[:, 2]
    kmax = int(np.abs(k).max())
    ks = np.arange(-kmax, kmax + 1)
    M = len(ks)
    Dsc = np.diag(0.5 * (2 * np.pi * ks / 15.0) ** 2).astype(np.complex128)
    Vs = []
    for s, vj in zip(shifts, v):
        V = np.zeros((M, M), dtype=np.complex128)
        for a in range(M):
            for b in range(M):
                if abs(ks[a] - ks[b]) == s:
                    V[a, b] = vj
        Vs.append(V)
    kappa, tau, nsteps = 0.0, 0.02, 20
    Hs = [(1.0 - kappa) / 3 * Dsc + V for V in Vs]
    E = lambda A, t: scipy.linalg.expm(-1j * t * A)  # noqa: E731
    Ssc = E(Hs[0], tau / 2) @ E(Hs[1], tau / 2) @ E(Hs[2], tau) @ E(Hs[1], tau / 2) @ E(Hs[0], tau / 2)
    # lifted-decaying data
    G = [2 * np.pi / 1.0, 2 * np.pi / 1.5, 2 * np.pi / 1.25]
    own2 = sum((G[j] * O.mn[:, j]) ** 2 for j in range(3))
    c = np.exp(-0.5 * (O.K[:, 0] - 1.0) ** 2 - 0.15 * own2).astype(np.complex128)
    c /= np.linalg.norm(c)

    def project(x):
        out = np.zeros(M, dtype=np.complex128)
        np.add.at(out, k + kmax, x)
        return out

    plan = ml.MultiSplitPlan(O, kappa)
    x = plan.evolve(c, tau, nsteps, "strang")
    ref = np.linalg.matrix_power(Ssc, nsteps) @ project(c)
    assert rel(project(x), ref) < 1e-9


def test_three_layer_unitarity_reversibility_and_free_particle():
    O = three_chain(100.0)
    c0 = wl.random_state(O.N, 2, seed=4)
    for kappa in (0.0, 0.4):
        plan = ml.MultiSplitPlan(O, kappa)
        c = plan.evolve(c0, 0.02, 25)
        assert np.abs(np.linalg.norm(c, axis=0) - np.linalg.norm(c0, axis=0)).max() < 1e-12
        back = ml.MultiSplitPlan(O, kappa).evolve(c, -0.02, 25)
        assert rel(back, c0) < 1e-12
    free = three_chain(100.0, v=(0.0, 0.0, 0.0))
    plan = ml.MultiSplitPlan(free, 0.3)
    c = plan.evolve(c0, 0.02, 10)
    assert rel(c, c0 * np.exp(-1j * 0.2 * 0.5 * free.K2)[:, None]) < 1e-13


def test_three_layer_product_set_counts():
    """Product cutoff: I = I_1 x I_2 x I_3, so every layer-j fibre has |I_j| rows."""
    O = three_chain(60.0, cutoff="product")
    sizes = []
    for j, Lj in enumerate((1.0, wl.GOLDEN, SQRT2)):
        g = 2 * np.pi / Lj
        sizes.append(sum(1 for m in range(-100, 101) if (g * m) ** 2 <= 120.0 * (1 + 1e-12)))
    assert O.N == sizes[0] * sizes[1] * sizes[2]
    for j in (1, 2, 3):
        assert {len(r) for _, r in O.fib[j]} == {sizes[j - 1]}


@pytest.mark.parametrize("flow,scheme", [("be", "lie"), ("cn", "strang")])
def test_rational_flows_reduce_to_the_two_layer_oracle(flow, scheme):
    spec = wl.twisted_system(120.0)
    O2 = splitting.Lifted.from_spec(spec)
    OL = ml.MultiLifted(spec.d, [spec.A1, spec.A2], spec.Ec, spec.cutoff, [spec.pot1, spec.pot2])
    c = wl.random_state(O2.N, 2, seed=6)
    for kappa in (0.0, 0.5):
        a = splitting.SplitPlan(O2, kappa, flow).evolve(c, 0.03, 3, scheme)
        b = ml.MultiSplitPlan(OL, kappa, flow).evolve(c, 0.03, 3, scheme)
        assert rel(b, a) < 1e-13


def smooth_state(K2, lift):
    """Data smooth in x and decaying in the lifted index: exp(-2 |K|^2 - 0.1 sum_j |G_j m_j|^2).
    Backward Euler reaches its O(tau) regime only once tau lambda << 1 on the excited modes, so
    the order pins use such data (as the two-layer pins use a Gaussian)."""
    c = np.exp(-2.0 * K2 - 0.1 * lift).astype(np.complex128)
    return c / np.linalg.norm(c)


@pytest.mark.parametrize("flow,scheme,order", [("be", "lie", 1.0), ("cn", "strang", 2.0)])
def test_three_layer_rational_flows(flow, scheme, order):
    """Backward Euler (Alg. 2) and Crank-Nicolson (eq. 4.6) sub-steps on three layers: one step
    equals the dense product of the same rational factors of the full lifted H_j (solves with
    the whole matrices), BE converges at order 1 and CN at order 2 against brute force
    (Thms 4.2, 4.3), CN keeps the mass exactly and BE never increases it (Thm 4.4, Sec. 5)."""
    O = three_chain(100.0)
    Dk, Hs = O.dense(0.0)
    I = np.eye(O.N)
    if flow == "be":
        R = lambda A, t: np.linalg.solve(I + 1j * t * A, I)  # noqa: E731
    else:
        R = lambda A, t: np.linalg.solve(I + 0.5j * t * A, I - 0.5j * t * A)  # noqa: E731
    tau = 0.05
    c = wl.random_state(O.N, 2, seed=5)
    plan = ml.MultiSplitPlan(O, 0.0, flow)
    H1, H2, H3 = Hs
    if scheme == "lie":
        M = R(H3, tau) @ R(H2, tau) @ R(H1, tau)
    else:
        M = R(H1, tau / 2) @ R(H2, tau / 2) @ R(H3, tau) @ R(H2, tau / 2) @ R(H1, tau / 2)
    assert rel(plan.evolve(c, tau, 1, scheme), M @ c) < 1e-12
    H = Dk + sum(Hs)
    lift = sum((O.mn[:, j:j + 1] @ O.Gs[j].T)[:, 0] ** 2 for j in range(3))
    c0 = smooth_state(O.K2, lift)
    T = 0.5
    exact = scipy.linalg.expm(-1j * T * H) @ c0
    Ks = (400, 800, 1600) if flow == "be" else (40, 80, 160)
    errs = [np.linalg.norm(plan.evolve(c0, T / K, K, scheme) - exact) for K in Ks]
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(s - order) < 0.1 for s in slopes), (errs, slopes)
    x = plan.evolve(c, 0.02, 30, scheme)
    drift = np.linalg.norm(x, axis=0) - np.linalg.norm(c, axis=0)
    if flow == "cn":
        assert np.abs(drift).max() < 1e-12
    else:
        assert drift.max() < 1e-14 and drift.min() < -1e-6


def test_example3_rational_flows():
    """The same rational schemes on the shared-block lift of Example 3: orders 1 (BE-Lie) and 2
    (CN-Strang) against brute force, CN mass exact."""
    from oracle import blocks
    O = blocks.example3(40.0)
    Dk, Hs = O.dense(0.0)
    H = Dk + sum(Hs)
    lift = np.zeros(O.N)
    for b, Rb in enumerate(O.Rs):
        g = O.mn[:, O.off[b]:O.off[b + 1]] @ Rb.T
        lift += (g * g).sum(axis=1)
    c0 = smooth_state(O.K2, lift)
    T = 0.5
    exact = scipy.linalg.expm(-1j * T * H) @ c0
    for flow, scheme, order, Ks in (("be", "lie", 1.0, (400, 800, 1600)), ("cn", "strang", 2.0, (40, 80, 160))):
        plan = ml.MultiSplitPlan(O, 0.0, flow)
        errs = [np.linalg.norm(plan.evolve(c0, T / K, K, scheme) - exact) for K in Ks]
        slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
        assert all(abs(s - order) < 0.1 for s in slopes), (flow, errs, slopes)
    c = wl.random_state(O.N, 1, seed=8)[:, 0]
    x = ml.MultiSplitPlan(O, 0.3, "cn").evolve(c, 0.02, 20, "strang")
    assert abs(np.linalg.norm(x) - np.linalg.norm(c)) < 1e-12
