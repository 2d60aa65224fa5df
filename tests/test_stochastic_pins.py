"""Pins of the semi-implicit / random batch steps (Alg. 1, Alg. 4) and of stochastic layer
splitting with a learned proposal, against closed forms, dense brute force, exact enumeration of
the sampling distributions, and finite differences."""
import itertools

import numpy as np
import pytest
import scipy.linalg

from oracle import lifted, observables, reference, splitting
from oracle import stochastic as sto
from paper_2103_14897_amd import workloads as wl


@pytest.fixture(scope="module")
def tiny():
    w = wl.tiny_chain()
    O = splitting.Lifted.from_spec(w.spec)
    c = wl.random_state(O.N, 3, seed=4)
    return w, O, c


# ---------------------------------------------------------------- Alg. 1

def test_semi_implicit_equals_dense_definition(tiny):
    """Fibre-wise potentials equal the full lifted V^1, V^2 of eq. (3.6) in the Alg. 1 update."""
    w, O, c = tiny
    D, V1, V2 = lifted.dense_lifted(O.A1, O.A2, O.mn, O.pot1, O.pot2)
    tau = 0.02
    ref = np.linalg.solve(np.eye(O.N) + 1j * tau * D, c - 1j * tau * (V1 + V2) @ c)
    assert np.abs(sto.semi_implicit_step(O, c, tau) - ref).max() < 1e-14


def test_semi_implicit_free_particle_closed_form():
    """With both potentials zero each step divides mode i by (1 + i tau |K_i|^2 / 2)."""
    spec = wl.chain_system(200.0, v1=0.0, v2=0.0)
    O = splitting.Lifted.from_spec(spec)
    c = wl.random_state(O.N, 2, seed=1)
    tau, k = 0.01, 7
    x = c
    for _ in range(k):
        x = sto.semi_implicit_step(O, x, tau)
    ref = c / ((1.0 + 1j * tau * 0.5 * O.K2) ** k)[:, None]
    assert np.abs(x - ref).max() < 1e-14


def test_semi_implicit_first_order(tiny):
    """Thm 4.1: O(tau) error against exp(-i T H) of the full lifted matrix."""
    w, O, _ = tiny
    c0 = w.initial_state(O.mn)
    T = 0.4
    exact = reference.exact_flow(O, c0, T)
    errs = []
    for K in (400, 800, 1600):  # tau |K|^2 / 2 <= 0.2: the asymptotic range
        x = c0
        for _ in range(K):
            x = sto.semi_implicit_step(O, x, T / K)
        errs.append(np.linalg.norm(x.ravel() - exact.ravel()))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 1.0) < 0.15), rates


def test_semi_implicit_does_not_conserve_mass(tiny):
    """Sec. 5: unlike the exact-flow and Crank-Nicolson splittings, the semi-implicit step changes
    the mass (here by far more than rounding)."""
    w, O, _ = tiny
    x = w.initial_state(O.mn)
    for _ in range(50):
        x = sto.semi_implicit_step(O, x, 0.01)
    assert abs(observables.mass(x)[0] - 1.0) > 1e-6


# ---------------------------------------------------------------- Alg. 4

def test_subset_sampler_uniform_over_ordered_tuples():
    """Uniforms at the midpoints of an nf x (nf-1) x ... lattice produce every ordered tuple of
    distinct fibres exactly once."""
    nf, p = 6, 3
    grids = [(np.arange(nf - s) + 0.5) / (nf - s) for s in range(p)]
    seen = {}
    for us in itertools.product(*grids):
        u = np.array(us)[None, :]
        wt = sto.subset_weights(nf, p, u)
        chosen = tuple(sorted(np.flatnonzero(wt[:, 0])))
        assert len(chosen) == p and np.allclose(wt[list(chosen), 0], nf / p)
        seen[chosen] = seen.get(chosen, 0) + 1
    assert len(seen) == len(list(itertools.combinations(range(nf), p)))
    assert set(seen.values()) == {6}  # p! orderings of each subset


def test_random_batch_all_fibres_is_alg1(tiny):
    w, O, c = tiny
    n1, n2 = len(O.fib[1]), len(O.fib[2])
    u = wl.uniforms((3, max(n1, n2)), seed=2)
    x = sto.random_batch_step(O, c, 0.01, n1, u[:, :n1], n2, u[:, :n2])
    assert np.abs(x - sto.semi_implicit_step(O, c, 0.01)).max() < 1e-15


@pytest.mark.parametrize("p", [1, 2])
def test_random_batch_expectation_is_alg1(tiny, p):
    """Averaging Alg. 4 over every pair of equally likely subsets gives Alg. 1 exactly."""
    w, O, c = tiny
    n1, n2 = len(O.fib[1]), len(O.fib[2])
    tau = 0.02
    acc = np.zeros_like(c)
    S1 = list(itertools.combinations(range(n1), p))
    S2 = list(itertools.combinations(range(n2), p))
    for s1 in S1:
        a1 = np.zeros((n1, c.shape[1]))
        a1[list(s1)] = n1 / p
        for s2 in S2:
            a2 = np.zeros((n2, c.shape[1]))
            a2[list(s2)] = n2 / p
            acc += sto.semi_implicit_step(O, c, tau, a1, a2)
    acc /= len(S1) * len(S2)
    assert np.abs(acc - sto.semi_implicit_step(O, c, tau)).max() < 1e-13


# ---------------------------------------------------------------- proposal and sampling

def test_proposal_special_cases():
    rng = np.random.default_rng(0)
    z = rng.standard_normal((4, 9))
    q = sto.proposal(z, 9, 4, 0.05)
    assert np.allclose(q.sum(axis=1), 1.0) and q.min() >= 0.05 / 9 * (1 - 1e-12)
    assert np.allclose(sto.proposal(z, 9, 4, 1.0), 1.0 / 9)
    assert np.allclose(sto.proposal(np.full((4, 9), 3.7), 9, 4, 0.3), 1.0 / 9)
    # softmax invariance to a per-column shift
    assert np.allclose(sto.proposal(z + 5.0, 9, 4, 0.05), q)


def test_inverse_cdf_frequencies():
    """Uniforms on the midpoints of a grid of G cells hit fibre f in q_f G +- 1 cells."""
    rng = np.random.default_rng(1)
    q = sto.proposal(rng.standard_normal((1, 13)), 13, 1, 0.1)
    G = 20000
    u = ((np.arange(G) + 0.5) / G)[None, :]
    f = sto.draw(q, u)[0]
    counts = np.bincount(f, minlength=13)
    assert np.all(np.abs(counts - q[0] * G) <= 1.0 + 1e-9)
    assert np.all(np.diff(f) >= 0)


@pytest.mark.parametrize("layer", [1, 2])
def test_sampled_pass_moments_exact(tiny, layer):
    """Exact enumeration of one draw (p = 1): the mean is the deterministic layer pass, and the mean
    squared deviation is sum_f b_f / q_f - sum_f b_f per column; two draws halve it."""
    w, O, c = tiny
    plan = splitting.SplitPlan(O, 0.0)
    t = 0.05
    nf = len(O.fib[layer])
    W = c.shape[1]
    rng = np.random.default_rng(3)
    q = sto.proposal(rng.standard_normal((W, nf)), nf, W, 0.1)
    det = plan.apply_fibres(c, layer, t)
    b = sto.increments(plan, layer, t, c)
    for p in (1, 2):
        mean = np.zeros_like(c)
        msd = np.zeros(W)
        for fs in itertools.product(range(nf), repeat=p):
            prob = np.prod([q[:, f] for f in fs], axis=0)  # per column
            wt = np.zeros((nf, W))
            for f in fs:
                wt[f] += 1.0 / (p * q[:, f])
            out = sto.sampled_pass(plan, layer, t, c, wt)
            mean += prob[None, :] * out
            msd += prob * (np.abs(out - det) ** 2).sum(axis=0)
        assert np.abs(mean - det).max() < 1e-13
        pred = ((b / q).sum(axis=1) - b.sum(axis=1)) / p
        assert np.allclose(msd, pred, rtol=1e-10, atol=1e-16)


def test_stochastic_strang_unbiased_with_state_dependent_proposal(tiny):
    """Enumerating every draw of the three sub-steps (p = 1), with a proposal computed from the
    current state's features, averages to the deterministic Strang step."""
    w, O, c = tiny
    c = c[:, :1]
    plan = splitting.SplitPlan(O, 0.5)
    tau = 0.05
    rng = np.random.default_rng(5)
    coef = rng.standard_normal(sto.n_features(O.d))
    eps = 0.2

    def logits(layer, x):
        return sto.features(O, layer, x)[..., :] @ coef

    det = plan.strang_step(c, tau)
    subs = sto.substeps("strang", tau)

    def expect(k, x):
        if k == len(subs):
            return x
        layer, t, tph = subs[k]
        nf = len(O.fib[layer])
        q = sto.proposal(logits(layer, x), nf, 1, eps)
        acc = np.zeros_like(x)
        for f in range(nf):
            wt = np.zeros((nf, 1))
            wt[f, 0] = 1.0 / q[0, f]
            y = sto.sampled_pass(plan, layer, t, x, wt)
            if tph != 0.0:
                y = plan.apply_phase(y, tph)
            acc += q[0, f] * expect(k + 1, y)
        return acc

    assert np.abs(expect(0, c) - det).max() < 1e-13


def test_stochastic_step_with_all_weight_on_every_fibre_is_deterministic(tiny):
    """p draws that cover every fibre once with q uniform reproduce the deterministic step."""
    w, O, c = tiny
    plan = splitting.SplitPlan(O, 0.0)
    nf = max(len(O.fib[1]), len(O.fib[2]))
    # uniforms at fibre midpoints: with q uniform, draw s lands on fibre s
    for layer in (1, 2):
        n = len(O.fib[layer])
        u = np.tile(((np.arange(n) + 0.5) / n)[None, :], (c.shape[1], 1))
        q = sto.proposal(None, n, c.shape[1], 0.0)
        assert np.array_equal(sto.draw(q, u)[0], np.arange(n))
        wt = sto.draw_weights(q, u)
        assert np.allclose(wt, 1.0)
        x = sto.sampled_pass(plan, layer, 0.03, c, wt)
        assert np.abs(x - plan.apply_fibres(c, layer, 0.03)).max() < 1e-14
    del nf


# ---------------------------------------------------------------- features

@pytest.mark.parametrize("spec", [wl.chain_system(200.0), wl.twisted_system(60.0)], ids=["1d", "2d"])
def test_features_shift_and_mass(spec):
    """shift + own wavevector = lifted wavevector K on every row of a fibre; the mass feature is
    log10 of the fibre's partial mass."""
    O = splitting.Lifted.from_spec(spec)
    c = wl.random_state(O.N, 2, seed=0)
    d = O.d
    kmax = np.sqrt(2.0 * O.Ec)
    G1 = 2.0 * np.pi * np.linalg.inv(O.A1).T
    G2 = 2.0 * np.pi * np.linalg.inv(O.A2).T
    for layer in (1, 2):
        X = sto.features(O, layer, c)
        assert X.shape == (2, len(O.fib[layer]), d + 3)
        for f, (_, rows) in enumerate(O.fib[layer]):
            own = O.mn[rows, :d] @ G1.T if layer == 1 else O.mn[rows, d:] @ G2.T
            assert np.allclose(own + X[0, f, :d] * kmax, O.K[rows], atol=1e-9)
            assert np.isclose(X[0, f, d], (X[0, f, :d] ** 2).sum())
            m = (np.abs(c[rows]) ** 2).sum(axis=0)
            assert np.allclose(10.0 ** (10.0 * X[:, f, d + 1]), m, rtol=1e-12)
        assert np.all(X[..., d + 2] == (-1.0 if layer == 1 else 1.0))


# ---------------------------------------------------------------- MLP, objective, optimiser

def test_mlp_backward_matches_finite_differences():
    nin, H = 5, 64
    theta = wl.mlp_init(nin, H, seed=3).astype(np.float64)
    theta += 0.05 * np.random.default_rng(0).standard_normal(theta.size)
    X = np.random.default_rng(1).standard_normal((17, nin))
    dz = np.random.default_rng(2).standard_normal(17)
    g = sto.mlp_backward(theta, X, dz, H)
    h = 1e-6
    fd = np.empty_like(theta)
    for k in range(theta.size):
        e = np.zeros_like(theta)
        e[k] = h
        fd[k] = (sto.mlp_forward(theta + e, X, H) @ dz - sto.mlp_forward(theta - e, X, H) @ dz) / (2 * h)
    assert np.abs(g - fd).max() < 1e-7 * max(1.0, np.abs(fd).max())


def test_mlp_forward_small_network_by_hand():
    """A 1-input, width-2 network evaluated term by term."""
    theta = np.array([0.3, -0.7,  0.1, 0.2,  0.5, -1.1, 0.4, 0.9,  -0.2, 0.3,  1.5, -2.0,  0.25])
    x = 0.8
    h1 = np.tanh(np.array([0.3 * x + 0.1, -0.7 * x + 0.2]))
    h2 = np.tanh(np.array([0.5 * h1[0] + 0.4 * h1[1] - 0.2, -1.1 * h1[0] + 0.9 * h1[1] + 0.3]))
    z = 1.5 * h2[0] - 2.0 * h2[1] + 0.25
    assert np.isclose(sto.mlp_forward(theta, np.array([[x]]), H=2)[0], z, rtol=1e-15)


def test_proposal_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    gptr = np.array([0, 7, 7 + 11, 7 + 11 + 5, 7 + 11 + 5 + 3])
    M = gptr[-1]
    z = rng.standard_normal(M)
    b = rng.random(M) ** 3
    b[gptr[3]:gptr[4]] = 0.0  # an empty group is skipped
    L, dz, lg = sto.proposal_loss(z, b, gptr, 0.07)
    assert lg[3] == 0.0
    h = 1e-6
    for k in range(M):
        e = np.zeros(M)
        e[k] = h
        fd = (sto.proposal_loss(z + e, b, gptr, 0.07)[0] - sto.proposal_loss(z - e, b, gptr, 0.07)[0]) / (2 * h)
        assert abs(dz[k] - fd) < 1e-7 * max(1.0, abs(fd))


def test_proposal_loss_optimum_and_uniform_value():
    """Cauchy-Schwarz: the objective is >= 1, equal to 1 with zero gradient at q ~ sqrt(b) (eps = 0);
    the uniform proposal gives n sum b / (sum sqrt b)^2."""
    rng = np.random.default_rng(6)
    b = rng.random(23) ** 4 + 1e-12
    gptr = np.array([0, 23])
    L, dz, _ = sto.proposal_loss(0.5 * np.log(b), b, gptr, 0.0)
    assert abs(L - 1.0) < 1e-12 and np.abs(dz).max() < 1e-12
    for _ in range(5):
        assert sto.proposal_loss(rng.standard_normal(23), b, gptr, 0.0)[0] > 1.0
    Lu = sto.proposal_loss(np.zeros(23), b, gptr, 0.0)[0]
    assert np.isclose(Lu, 23 * b.sum() / np.sqrt(b).sum() ** 2, rtol=1e-13)


def test_proposal_loss_is_the_sampled_pass_variance(tiny):
    """With targets b from the increments, p * E||S c - F c||^2 + sum b equals l * (sum sqrt b)^2."""
    w, O, c = tiny
    plan = splitting.SplitPlan(O, 0.0)
    layer, t = 2, 0.05
    nf = len(O.fib[layer])
    b = sto.increments(plan, layer, t, c[:, :1])[0]
    z = np.random.default_rng(7).standard_normal(nf)
    q = sto.proposal(z[None, :], nf, 1, 0.1)[0]
    det = plan.apply_fibres(c[:, :1], layer, t)
    msd = 0.0
    for f in range(nf):
        wt = np.zeros((nf, 1))
        wt[f, 0] = 1.0 / q[f]
        msd += q[f] * (np.abs(sto.sampled_pass(plan, layer, t, c[:, :1], wt) - det) ** 2).sum()
    L = sto.proposal_loss(z, b, np.array([0, nf]), 0.1)[0]
    assert np.isclose(msd + b.sum(), L * np.sqrt(b).sum() ** 2, rtol=1e-10)


def test_adam_constant_gradient_steps():
    """With a constant gradient the bias-corrected moments equal g and g^2 at every step, so each
    update is -lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    theta = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    for t in range(1, 8):
        new, m, v = sto.adam_step(theta, m, v, g, t, lr=0.01)
        assert np.allclose(new - theta, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)
        theta = new


def test_scipy_expm_reference_still_unitary(tiny):
    """Guard for the brute-force reference used above."""
    w, O, _ = tiny
    D, V1, V2 = lifted.dense_lifted(O.A1, O.A2, O.mn, O.pot1, O.pot2)
    U = scipy.linalg.expm(-1j * 0.1 * (D + V1 + V2))
    assert np.abs(U.conj().T @ U - np.eye(O.N)).max() < 1e-13
