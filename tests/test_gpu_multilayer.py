"""GPU parity of layer splitting for three layers against the L-layer oracle: propagators of
every layer and slot, Lie, Strang and Yoshida trajectories (FP64 <= 2e-12 relative L2 per
step; Yoshida 6e-12 per step for its three Strang steps), the
fused kinetic phase for kappa in {0, 0.4, 1}, single passes at ragged W in every precision,
single passes of the twisted trilayer at the benchmark's full size on sampled fibres,
mixed precision after many steps, mass, energy and per-layer fibre masses, two layers through
the layered constructor, and the entry points that take two-layer systems only (samplers and
the semi-implicit step)."""
import numpy as np
import pytest

from oracle import multilayer as ml
from oracle import splitting
from paper_2103_14897_amd import lsx
from paper_2103_14897_amd import workloads as wl

pytestmark = pytest.mark.gpu

CASES = {"chain3": lambda: wl.chain_layers(2000.0), "twisted3": lambda: wl.twisted_layers(250.0)}


def colrel(a, b):
    return (np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)).max()


def build(spec):
    S = lsx.System.layers(spec.d, spec.As, spec.Ec, spec.cutoff, spec.pots)
    O = ml.MultiLifted(spec.d, spec.As, spec.Ec, spec.cutoff, spec.pots)
    assert S.N == O.N and S.nlayers == 3
    return S, O


@pytest.mark.parametrize("which", sorted(CASES))
@pytest.mark.parametrize("kappa", [0.0, 1.0])
def test_three_layer_propagators(which, kappa):
    spec = CASES[which]()
    print(f"[case] propagators {which} kappa={kappa}", flush=True)
    S, O = build(spec)
    plan = ml.MultiSplitPlan(O, kappa)
    tau = 0.01
    P = lsx.Plan(S, tau, "strang", kappa, "fp64")
    try:
        slots = {1: {0: tau, 1: tau / 2}, 2: {1: tau / 2}, 3: {0: tau}}
        for layer, ts in slots.items():
            nf = S.nfibres[layer]
            for slot, t in ts.items():
                ref = plan.propagators(layer, t)
                for f in (0, nf // 3, nf // 2, nf - 1):
                    assert np.abs(P.propagator(layer, slot, f) - ref[f]).max() < 1e-13, (layer, slot, f)
        with pytest.raises(lsx.LsxError):
            P.propagator(2, 0, 0)  # layer 2 holds only tau/2 in the three-layer Strang plan
    finally:
        P.destroy()
        S.destroy()


@pytest.mark.parametrize("which", sorted(CASES))
@pytest.mark.parametrize("scheme,kappa", [("strang", 0.0), ("strang", 0.4), ("strang", 1.0), ("lie", 0.0),
                                          ("lie", 0.4), ("yoshida4", 0.0), ("yoshida4", 0.4)])
def test_three_layer_trajectories(which, scheme, kappa):
    spec = CASES[which]()
    print(f"[case] trajectory {which} {scheme} kappa={kappa}", flush=True)
    S, O = build(spec)
    plan = ml.MultiSplitPlan(O, kappa)
    W, tau = 5, 0.01
    per_step = 6e-12 if scheme == "yoshida4" else 2e-12
    P = lsx.Plan(S, tau, scheme, kappa, "fp64")
    st = lsx.State(P, W)
    try:
        c = wl.random_state(S.N, W, seed=7)
        for nsteps in (1, 4):
            st.upload(c)
            st.step(nsteps)
            ref = plan.evolve(c, tau, nsteps, scheme)
            assert colrel(st.download(), ref) < per_step * nsteps, nsteps
        # split calls compose: 2 + 2 steps equal 4 steps
        st.upload(c)
        st.step(2)
        st.step(2)
        assert colrel(st.download(), plan.evolve(c, tau, 4, scheme)) < 4 * per_step
    finally:
        st.destroy()
        P.destroy()
        S.destroy()


@pytest.mark.parametrize("W", [1, 15, 33, 130])
@pytest.mark.parametrize("precision", ["fp64", "mix_fp32", "mix_bf16x3"])
def test_three_layer_single_passes(W, precision):
    spec = wl.chain_layers(2000.0)
    S, O = build(spec)
    plan = ml.MultiSplitPlan(O, 0.0)
    tau = 0.01
    P = lsx.Plan(S, tau, "strang", 0.0, precision)
    st = lsx.State(P, W)
    try:
        c = wl.random_state(S.N, W, seed=W)
        tol = 1e-12 if precision == "fp64" else 1e-7
        for layer, slot, t in ((1, 1, tau / 2), (2, 1, tau / 2), (3, 0, tau)):
            st.upload(c)
            st.fibre_pass(layer, slot)
            assert colrel(st.download(), plan.apply_fibres(c, layer, t)) < tol, (layer, st.tuning(layer))
    finally:
        st.destroy()
        P.destroy()
        S.destroy()


def test_three_layer_mixed_precision_long_run():
    spec = wl.twisted_layers(250.0)
    S, O = build(spec)
    W, tau = 8, 5e-3
    c = wl.random_state(S.N, W, seed=3)
    out = {}
    try:
        for prec in ("fp64", "mix_fp32", "mix_bf16x3"):
            P = lsx.Plan(S, tau, "strang", 0.5, prec)
            st = lsx.State(P, W)
            st.upload(c)
            st.step(60)
            out[prec] = st.download()
            st.destroy()
            P.destroy()
        for prec in ("mix_fp32", "mix_bf16x3"):
            err = colrel(out[prec], out["fp64"])
            print(f"  {prec}: 60 steps rel err vs FP64 {err:.2e}")
            assert err < 1e-6
        assert np.abs(np.linalg.norm(out["fp64"], axis=0) - np.linalg.norm(c, axis=0)).max() < 1e-11
    finally:
        S.destroy()


def test_three_layer_observables():
    """Mass, energy Re c^H (D + V^1 + V^2 + V^3) c from the oracle's dense operators, and the
    partial masses of every layer's fibres."""
    spec = wl.chain_layers(150.0)
    S, O = build(spec)
    D, Vs = O.dense(1.0)  # kappa = 1: H_j = V^j
    H = D + sum(Vs)
    W = 3
    P = lsx.Plan(S, 0.01, "strang", 0.0, "fp64")
    st = lsx.State(P, W)
    try:
        c = wl.random_state(S.N, W, seed=11) * np.array([1.0, 2.0, 0.5])[None, :]
        st.upload(c)
        mask = lsx.OBS_MASS | lsx.OBS_ENERGY | lsx.OBS_FIBRE_MASS_1 | lsx.OBS_FIBRE_MASS_2 | lsx.OBS_FIBRE_MASS_3
        r = st.observables(mask)
        m = (np.abs(c) ** 2).sum(axis=0)
        E = np.real(np.einsum("iw,ij,jw->w", c.conj(), H, c))
        assert np.abs(r["mass"] - m).max() < 1e-13 * m.max()
        assert np.abs(r["energy"] - E).max() < 1e-12 * np.abs(E).max()
        for layer in (1, 2, 3):
            ref = np.array([(np.abs(c[rows]) ** 2).sum(axis=0) for _, rows in O.fib[layer]])
            assert np.abs(r[f"fibre_mass_{layer}"] - ref).max() < 1e-13 * m.max(), layer
    finally:
        st.destroy()
        P.destroy()
        S.destroy()


def test_two_layers_through_layers_constructor_bit_identical(monkeypatch):
    # one forced tile shape for both states: the autotuner may otherwise pick shapes with
    # different summation orders
    monkeypatch.setenv("LSX_NB", "1")
    monkeypatch.setenv("LSX_KS", "2")
    spec = wl.chain_system(2000.0)
    A = lsx.System.from_spec(spec)
    B = lsx.System.layers(spec.d, [spec.A1, spec.A2], spec.Ec, spec.cutoff, [spec.pot1, spec.pot2])
    out = []
    try:
        for S in (A, B):
            P = lsx.Plan(S, 0.01, "strang", 0.3, "fp64")
            st = lsx.State(P, 6)
            st.upload(wl.random_state(S.N, 6, seed=5))
            st.step(5)
            out.append(st.download())
            st.destroy()
            P.destroy()
        assert np.array_equal(out[0], out[1])
    finally:
        A.destroy()
        B.destroy()


@pytest.mark.parametrize("which", sorted(CASES))
@pytest.mark.parametrize("scheme,flow,kappa", [("lie_be", "be", 0.0), ("lie_be", "be", 0.4),
                                               ("strang_cn", "cn", 0.0), ("strang_cn", "cn", 0.4)])
def test_three_layer_rational_trajectories(which, scheme, flow, kappa):
    """Backward-Euler Lie and Crank-Nicolson Strang on three layers against the oracle's linear
    solves (FP64 <= 2e-12 relative L2 per step); CN keeps the mass, BE decreases it."""
    spec = CASES[which]()
    print(f"[case] rational {which} {scheme} kappa={kappa}", flush=True)
    S, O = build(spec)
    plan = ml.MultiSplitPlan(O, kappa, flow)
    comp = "lie" if flow == "be" else "strang"
    W, tau = 4, 0.01
    P = lsx.Plan(S, tau, scheme, kappa, "fp64")
    st = lsx.State(P, W)
    try:
        c = wl.random_state(S.N, W, seed=12)
        for nsteps in (1, 4):
            st.upload(c)
            st.step(nsteps)
            assert colrel(st.download(), plan.evolve(c, tau, nsteps, comp)) < 2e-12 * nsteps, nsteps
        m = st.observables(lsx.OBS_MASS)["mass"]
        if flow == "cn":
            assert np.abs(m - 1.0).max() < 1e-12
        else:
            assert m.max() < 1.0
    finally:
        st.destroy()
        P.destroy()
        S.destroy()


def test_three_layer_yoshida_slots():
    spec = wl.twisted_layers(150.0)
    S, O = build(spec)
    g1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
    g0 = 1.0 - 2.0 * g1
    tau = 0.01
    plan = ml.MultiSplitPlan(O, 0.3)
    P = lsx.Plan(S, tau, "yoshida4", 0.3, "fp64")
    try:
        slots = {1: {0: g1 * tau, 1: g1 * tau / 2, 2: (g1 + g0) * tau / 2}, 2: {0: g1 * tau / 2, 1: g0 * tau / 2},
                 3: {0: g1 * tau, 2: g0 * tau}}
        for layer, ts in slots.items():
            for slot, t in ts.items():
                ref = plan.propagators(layer, t)
                for f in (0, S.nfibres[layer] // 2, S.nfibres[layer] - 1):
                    assert np.abs(P.propagator(layer, slot, f) - ref[f]).max() < 1e-13, (layer, slot, f)
        with pytest.raises(lsx.LsxError):
            P.propagator(3, 1, 0)
    finally:
        P.destroy()
        S.destroy()


def test_three_layer_rejections():
    spec = wl.chain_layers(150.0)
    S, _ = build(spec)
    try:
        P = lsx.Plan(S, 0.01, "strang", 0.0, "fp64")
        st = lsx.State(P, 2)
        try:
            with pytest.raises(lsx.LsxError):
                st.si_step(1)
            with pytest.raises(lsx.LsxError):
                lsx.Sampler(st, 2, 2)
            with pytest.raises(lsx.LsxError):
                st.fibre_pass(4, 0)
        finally:
            st.destroy()
            P.destroy()
    finally:
        S.destroy()


@pytest.mark.parametrize("precision", ["fp64", "mix_fp32", "mix_bf16x3"])
def test_trilayer_full_size_sampled_passes(precision):
    """The twisted trilayer at the size the benchmark runs (Ec = 1000, N = 415135, 9061 fibres
    per layer, W = 128, tau = 5e-3, Strang) in the tuned launch configuration: single passes
    of every layer (the slots the Strang step uses: tau for layers 1 and 3, tau / 2 for layer
    2) on sampled fibres (the longest, the shortest and two at random) against the oracle's
    propagator of each fibre, built from the oracle's own row lists."""
    print(f"[case] trilayer full size sampled passes {precision}", flush=True)
    S, O = build(wl.twisted_layers(1000.0))
    assert S.N == 415135 and np.array_equal(S.index(), O.mn)
    tau, W = 5e-3, 128
    P = lsx.Plan(S, tau, "strang", 0.0, precision)
    st = lsx.State(P, W)
    rng = np.random.default_rng(6)
    tol = 1e-12 if precision == "fp64" else 1e-7
    try:
        c = wl.random_state(S.N, W, seed=23)
        for layer, slot in ((1, 0), (2, 1), (3, 0)):
            t = tau if slot == 0 else tau / 2
            rows_all = [rows for _, rows in O.fib[layer]]
            L = np.array([len(r) for r in rows_all])
            picks = sorted({int(np.argmax(L)), int(np.argmin(L))} | {int(x) for x in rng.integers(len(L), size=2)})
            st.upload(c)
            st.fibre_pass(layer, slot)
            got = st.download()
            for f in picks:
                r = rows_all[f]
                Pf = splitting.propagator_from_hamiltonian(O.fibre_hamiltonian(layer, r, 0.0), t)
                err = colrel(got[r], Pf @ c[r])
                assert err < tol, (precision, layer, f, len(r), err, st.tuning(layer))
    finally:
        st.destroy()
        P.destroy()
        S.destroy()


def test_trilayer_full_size_mixed_within_1e6_of_fp64():
    """The twisted trilayer at the benchmark's size (Ec = 1000, N = 415135, W = 128, Strang
    tau = 5e-3): after 50 steps from the same random unit wavepackets, the FP32 and BF16x3 paths
    are within 1e-6 relative L2 of the FP64 path (max over wavepackets), and every mass stays
    within the paths' bounds."""
    spec = wl.twisted_layers(1000.0)
    S = lsx.System.layers(spec.d, spec.As, spec.Ec, spec.cutoff, spec.pots)
    c0 = wl.random_state(S.N, 128, seed=0)
    out = {}
    try:
        for prec in ("fp64", "mix_fp32", "mix_bf16x3"):
            print(f"[case] trilayer full size 50 steps {prec}", flush=True)
            P = lsx.Plan(S, 5e-3, "strang", 0.0, prec)
            st = lsx.State(P, 128)
            try:
                st.upload(c0)
                st.step(50)
                out[prec] = st.download()
                m = st.observables(lsx.OBS_MASS)["mass"]
                assert np.abs(m - 1.0).max() < (1e-13 * 50 if prec == "fp64" else 1e-6), prec
            finally:
                st.destroy()
                P.destroy()
        for prec in ("mix_fp32", "mix_bf16x3"):
            err = colrel(out[prec], out["fp64"])
            print(f"  {prec}: rel L2 vs FP64 after 50 steps {err:.2e}", flush=True)
            assert err <= 1e-6, (prec, err)
    finally:
        S.destroy()
