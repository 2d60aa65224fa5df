"""Propagator sharing over point symmetries (rotations of the plane, or x -> -x in 1D, that map
every layer's reciprocal lattice, potential and the lifted index set onto themselves): the plan
stores one propagator per orbit of fibres, every fibre's propagator still equals the oracle's,
and whole trajectories agree with the unshared plan (LSX_SYMMETRY=0) and with the oracle."""
import numpy as np
import pytest

from oracle import splitting
from paper_2103_14897_amd import lsx
from paper_2103_14897_amd import workloads as wl

pytestmark = pytest.mark.gpu


def colrel(a, b):
    return (np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)).max()


def orbit_count(O, M, layer):
    """Number of orbits of layer `layer`'s fibres under the symmetries M [nsym, 2, d, d],
    computed from the oracle's own index set and fibres."""
    d = O.d
    keys = {tuple(r): i for i, r in enumerate(O.mn.tolist())}
    fib_of = np.empty(O.N, dtype=np.int64)
    for f, (_, rows) in enumerate(O.fib[layer]):
        fib_of[rows] = f
    seen = np.zeros(len(O.fib[layer]), dtype=bool)
    n = 0
    for f, (_, rows) in enumerate(O.fib[layer]):
        if seen[f]:
            continue
        n += 1
        seen[f] = True
        r = O.mn[rows[0]]
        for Mg in M:
            img = np.concatenate([Mg[0] @ r[:d], Mg[1] @ r[d:]])
            seen[fib_of[keys[tuple(int(x) for x in img)]]] = True
    return n


@pytest.mark.parametrize("spec,kappa", [(wl.chain_system(2.0e4), 0.0), (wl.twisted_system(1500.0), 0.0),
                                        (wl.twisted_system(900.0), 0.5)], ids=["chain", "twisted", "twisted-k05"])
def test_shared_propagators_and_trajectories(monkeypatch, spec, kappa):
    print(f"[case] symmetry sharing {spec.name} kappa={kappa}", flush=True)
    S = lsx.System.from_spec(spec)
    O = splitting.Lifted.from_spec(spec)
    assert np.array_equal(S.index(), O.mn)
    M = S.symmetries().astype(np.int64)
    tau, W, K = 0.005, 16, 6
    P = lsx.Plan(S, tau, "strang", kappa, "fp64")
    monkeypatch.setenv("LSX_SYMMETRY", "0")
    P0 = lsx.Plan(S, tau, "strang", kappa, "fp64")
    monkeypatch.delenv("LSX_SYMMETRY")
    try:
        plan = splitting.SplitPlan(O, kappa)
        for layer in (1, 2):
            nd, ns = P.sharing(layer)
            assert ns == len(M) >= 1
            assert nd == orbit_count(O, M, layer) < S.nfibres[layer]
            assert P0.sharing(layer) == (S.nfibres[layer], 0)
            ref = plan.propagators(layer, tau)
            nf = S.nfibres[layer]
            for f in sorted(set([0, 1, nf // 3, nf // 2, nf - 2, nf - 1])):
                assert np.abs(P.propagator(layer, 0, f) - ref[f]).max() < 1e-13, (layer, f)
        c0 = wl.random_state(S.N, W, seed=2)
        out = {}
        for name, pl in (("shared", P), ("unshared", P0)):
            st = lsx.State(pl, W)
            st.upload(c0)
            st.step(K)
            out[name] = st.download()
            st.upload(c0)
            st.fibre_pass(2, 0)  # the last layer's own pass from and to canonical order
            out[name + "_f2"] = st.download()
            st.destroy()
        assert colrel(out["shared"], out["unshared"]) < 1e-13
        assert colrel(out["shared"], plan.evolve(c0, tau, K)) < 1e-12 * K
        assert colrel(out["shared_f2"], plan.apply_fibres(c0, 2, tau)) < 1e-13
        assert colrel(out["shared_f2"], out["unshared_f2"]) < 1e-13
    finally:
        P.destroy()
        P0.destroy()
        S.destroy()


@pytest.mark.parametrize("precision", ["mix_fp32", "mix_bf16x3"])
def test_shared_mixed_passes_and_w1(precision):
    """Mixed formats (shared off-diagonal part and FP64 diagonal) and the single-wavepacket
    passes with shared propagators, against the oracle."""
    spec = wl.twisted_system(900.0)
    print(f"[case] symmetry sharing mixed {precision}", flush=True)
    S = lsx.System.from_spec(spec)
    O = splitting.Lifted.from_spec(spec)
    plan = splitting.SplitPlan(O, 0.0)
    P = lsx.Plan(S, 0.005, "strang", 0.0, precision)
    try:
        assert P.sharing(1)[0] < S.nfibres[1]
        for W in (1, 20):
            c = wl.random_state(S.N, W, seed=W)
            st = lsx.State(P, W)
            st.upload(c)
            st.step(3)
            got = st.download()
            st.destroy()
            assert colrel(got, plan.evolve(c, 0.005, 3)) < 1e-7, W
    finally:
        P.destroy()
        S.destroy()


def test_shared_batch_mixes_shared_and_unshared_systems():
    """A batch of a symmetric chain (last layer reordered), a chain whose complex potential has no
    symmetry (last layer in canonical order) and a twisted bilayer: the batched passes gather
    through the identity where a system needs no table; every system equals its own oracle."""
    asym = {(1,): 0.6 + 0.45j, (-1,): 0.6 - 0.45j}
    specs = [(wl.chain_system(971.0), 8), (wl.chain_system(971.0, pot1=asym), 8), (wl.twisted_system(400.0), 16)]
    print("[case] batch of shared and unshared systems", flush=True)
    made = []
    try:
        for spec, W in specs:
            S = lsx.System.from_spec(spec)
            P = lsx.Plan(S, 0.004, "strang", 0.0, "fp64")
            c0 = wl.random_state(S.N, W, seed=W)
            st = lsx.State(P, W)
            st.upload(c0)
            O = splitting.Lifted.from_spec(spec)
            made.append((S, P, st, c0, splitting.SplitPlan(O, 0.0).evolve(c0, 0.004, 5)))
        assert made[0][1].sharing(2)[1] == 1 and made[1][1].sharing(2)[1] == 0
        B = lsx.Batch([m[2] for m in made])
        for _ in range(2):
            for S, P, st, c0, ref in made:
                st.upload(c0)
            B.step(5)
            for S, P, st, c0, ref in made:
                assert colrel(st.download(), ref) < 5e-12
        B.destroy()
    finally:
        for S, P, st, c0, ref in made:
            st.destroy()
            P.destroy()
            S.destroy()
