"""Batched uneven systems: one grouped launch per pass over several systems.

Each system stepped inside a batch must equal the oracle's unmerged evolution of that
system (FP64: <= 1e-12 per step; mixed: the rounding bound derived in mixed_bounds.py) and
the same system stepped on its own (up to the summation order of a different tile shape),
for every scheme and precision, with systems of different lattices, cutoffs, dimensions and
wavepacket counts; the replayed HIP graph of the step body must give the same result on
every call.  The short runs here set LSX_GRAPH_PASSES=2 (graphs of one body repetition), so
that they replay graphs (LSX_GRAPH=1: whatever the pass times); test_default_graphs_equal_eager_launches
runs the default graph size.
"""
import math

import numpy as np
import pytest

import mixed_bounds
from oracle import blocks
from oracle import multilayer as ml
from oracle import splitting
from paper_2103_14897_amd import lsx
from paper_2103_14897_amd import workloads as wl

pytestmark = pytest.mark.gpu


def colrel(a, b):
    return (np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)).max()


@pytest.fixture(autouse=True)
def one_body_graphs(monkeypatch):
    monkeypatch.setenv("LSX_GRAPH", "1")
    monkeypatch.setenv("LSX_GRAPH_PASSES", "2")


def systems():
    return [
        (wl.chain_system(971.0), 8),
        (wl.chain_system(2000.0, L2=math.sqrt(2.0)), 16),
        (wl.chain_system(500.0, L2=math.sqrt(3.0)), 4),
        (wl.twisted_system(600.0, theta_deg=3.0), 16),
        (wl.twisted_system(400.0, theta_deg=5.0), 24),
    ]


@pytest.mark.parametrize("scheme", ["strang", "lie", "strang_cn"])
@pytest.mark.parametrize("precision,kappa", [("fp64", 0.0), ("mix_fp32", 1.0), ("mix_bf16x3", 0.0)])
def test_batch_equals_individual(scheme, precision, kappa):
    print(f"[case] batch {scheme} {precision} kappa={kappa}", flush=True)
    tau, nsteps = 0.004, 7
    flow = "cn" if scheme == "strang_cn" else "exact"
    made = []
    for spec, W in systems():
        S = lsx.System.from_spec(spec)
        P = lsx.Plan(S, tau, scheme, kappa, precision)
        c0 = wl.random_state(S.N, W, seed=W)
        ref_st = lsx.State(P, W)
        ref_st.upload(c0)
        ref_st.step(nsteps)
        ref = ref_st.download()
        ref_st.destroy()
        # the oracle's unmerged evolution of the same system from the same data
        O = splitting.Lifted.from_spec(spec)
        assert np.array_equal(S.index(), O.mn)
        plan = splitting.SplitPlan(O, kappa, flow)
        oref = plan.evolve(c0, tau, nsteps, "lie" if scheme == "lie" else "strang")
        if precision == "fp64":
            bound = 0.0
        elif scheme == "lie":
            bound = mixed_bounds.sequence_bound(plan, mixed_bounds.lie_passes(tau, nsteps), precision)
        else:
            seq = mixed_bounds.strang_passes(tau, nsteps, merged=(flow == "exact"))
            bound = mixed_bounds.sequence_bound(plan, seq, precision)
        st = lsx.State(P, W)
        st.upload(c0)
        made.append((S, P, st, c0, ref, oref, bound))
    B = lsx.Batch([m[2] for m in made])
    fp64_tol = 1e-12 * nsteps
    for call in range(2):
        if call:
            # a second call replays the captured body graph from a fresh upload
            for m in made:
                m[2].upload(m[3])
        B.step(nsteps)
        for S, P, st, c0, ref, oref, bound in made:
            got = st.download()
            e_or, e_ind = colrel(got, oref), colrel(got, ref)
            print(f"  N={S.N} vs oracle {e_or:.2e} (bound {bound + fp64_tol:.2e}), vs individual {e_ind:.2e}")
            assert e_or <= bound + fp64_tol
            # batch and individual runs differ only in their tiles' summation order: each is
            # within `bound` of FP64 arithmetic (exactly equal orders in FP64: ~rounding)
            assert e_ind <= (2 * bound if precision != "fp64" else 1e-13)
    B.destroy()
    for S, P, st, c0, ref, oref, bound in made:
        st.destroy()
        P.destroy()
        S.destroy()


def test_batch_single_state_w1_and_errors():
    S = lsx.System.from_spec(wl.chain_system(971.0))
    P = lsx.Plan(S, 0.01, "strang", 0.0, "fp64")
    a, b = lsx.State(P, 1), lsx.State(P, 1)
    c = wl.random_state(S.N, 1, seed=2)
    a.upload(c)
    a.step(5)
    ref = a.download()
    b.upload(c)
    B = lsx.Batch([b])
    B.step(5)
    assert colrel(b.download(), ref) < 1e-14
    with pytest.raises(lsx.LsxError) as e:
        b.destroy()
    assert e.value.code == lsx.LSX_E_STATE
    c64 = lsx.State(P, 16)
    with pytest.raises(lsx.LsxError):
        lsx.Batch([a, c64])  # W = 1 and W > 1 cannot share a batch
    B.destroy()
    for o in (a, b, c64, P, S):
        o.destroy()


@pytest.mark.parametrize("precision", ["fp64", "mix_fp32", "mix_bf16x3"])
@pytest.mark.parametrize("w1", [False, True])
def test_persistent_launch_equals_one_workgroup_per_tile(monkeypatch, precision, w1):
    """Persistent batched launches (per-XCD tile queues on device counters that the last
    workgroup clears, or a static stride) compute every tile exactly as the
    one-workgroup-per-tile launch: with
    one forced tile shape the results agree bit for bit, over 40 steps of replayed graphs
    (a queue left uncleared would skip the tiles of the next launch)."""
    print(f"[case] persistent batch {precision} w1={w1}", flush=True)
    monkeypatch.setenv("LSX_NB", "1")
    monkeypatch.setenv("LSX_KS", "2")
    out = {}
    for persist in ("1", "2", "0"):
        monkeypatch.setenv("LSX_PERSIST", persist)
        made = []
        for k, (spec, W) in enumerate(systems()):
            S = lsx.System.from_spec(spec)
            P = lsx.Plan(S, 0.004, "strang", 0.5, precision)
            W = 1 if w1 else W
            st = lsx.State(P, W)
            st.upload(wl.random_state(S.N, W, seed=k))
            made.append((S, P, st))
        B = lsx.Batch([m[2] for m in made])
        assert B.tuning(1)[3] == int(persist) and B.tuning(2)[3] == int(persist)
        B.step(1)
        B.step(39)
        out[persist] = [st.download() for _, _, st in made]
        B.destroy()
        for S, P, st in made:
            st.destroy()
            P.destroy()
            S.destroy()
    for mode in ("1", "2"):
        for a, b in zip(out[mode], out["0"]):
            assert np.array_equal(a, b), mode


@pytest.mark.parametrize("scheme", ["strang", "lie", "lie_be", "strang_cn", "yoshida4"])
def test_three_layer_batch_equals_individual(scheme):
    """Three-layer systems of different sizes in one batch: every system equals the same system
    stepped on its own and the L-layer oracle's unmerged evolution (FP64, 2e-12 per step,
    6e-12 for Yoshida's three Strang steps).  Three-layer Lie has an odd number of passes per step, so its graph
    holds two repetitions and an odd leftover runs eagerly (7 steps: head, 2 replays, 1 extra,
    tail)."""
    print(f"[case] three-layer batch {scheme}", flush=True)
    specs = [(wl.chain_layers(800.0), 8), (wl.chain_layers(1500.0, periods=(1.0, math.sqrt(2.0), math.sqrt(3.0))), 5),
             (wl.twisted_layers(120.0), 4)]
    made = []
    flow = {"lie_be": "be", "strang_cn": "cn"}.get(scheme, "exact")
    per_step = 6e-12 if scheme == "yoshida4" else 2e-12
    try:
        for spec, W in specs:
            S = lsx.System.layers(spec.d, spec.As, spec.Ec, spec.cutoff, spec.pots)
            P = lsx.Plan(S, 0.004, scheme, 0.3, "fp64")
            c0 = wl.random_state(S.N, W, seed=W)
            ref = lsx.State(P, W)
            ref.upload(c0)
            ref.step(7)
            st = lsx.State(P, W)
            st.upload(c0)
            O = ml.MultiLifted(spec.d, spec.As, spec.Ec, spec.cutoff, spec.pots)
            assert np.array_equal(S.index(), O.mn.astype(np.int32))
            oplan = ml.MultiSplitPlan(O, 0.3, flow)
            oref = oplan.evolve(c0, 0.004, 7, {"lie_be": "lie", "strang_cn": "strang"}.get(scheme, scheme))
            made.append((S, P, st, ref, c0, oref))
        B = lsx.Batch([m[2] for m in made])
        for _ in range(2):  # the second call replays the captured graph
            for S, P, st, ref, c0, oref in made:
                st.upload(c0)
            B.step(7)
            for S, P, st, ref, c0, oref in made:
                got = st.download()
                assert colrel(got, ref.download()) < 1e-13
                assert colrel(got, oref) < 7 * per_step
        B.destroy()
    finally:
        for S, P, st, ref, c0, oref in made:
            st.destroy()
            ref.destroy()
            P.destroy()
            S.destroy()


def test_example3_batch_and_mixed_layer_counts():
    made = []
    try:
        checks = []
        for k, Ec in enumerate((60.0, 100.0)):
            spec = wl.example3_system(Ec)
            S = lsx.System.blocks(spec.Rs, spec.groups, spec.Ec, spec.layers, spec.pots)
            P = lsx.Plan(S, 0.01, "strang", 0.0, "mix_fp32")
            c0 = wl.random_state(S.N, 16, seed=k)
            ref = lsx.State(P, 16)
            ref.upload(c0)
            ref.step(6)
            st = lsx.State(P, 16)
            st.upload(c0)
            made.append((S, P, st, ref))
            O = blocks.example3(Ec)
            assert np.array_equal(S.index(), O.mn.astype(np.int32))
            oplan = ml.MultiSplitPlan(O, 0.0)
            bound = mixed_bounds.sequence_bound(oplan, mixed_bounds.strang_passes(0.01, 6), "mix_fp32")
            checks.append((oplan.evolve(c0, 0.01, 6, "strang"), bound))
        B = lsx.Batch([m[2] for m in made])
        B.step(6)
        for (S, P, st, ref), (oref, bound) in zip(made, checks):
            got = st.download()
            assert colrel(got, oref) <= bound + 6 * 2e-12
            assert colrel(got, ref.download()) <= 2 * bound
        B.destroy()
        spec = wl.chain_layers(400.0)
        S3 = lsx.System.layers(spec.d, spec.As, spec.Ec, spec.cutoff, spec.pots)
        P3 = lsx.Plan(S3, 0.01, "strang", 0.0, "mix_fp32")
        s3 = lsx.State(P3, 16)
        try:
            with pytest.raises(lsx.LsxError):
                lsx.Batch([made[0][2], s3])  # two-layer and three-layer systems do not mix
        finally:
            s3.destroy()
            P3.destroy()
            S3.destroy()
    finally:
        for S, P, st, ref in made:
            st.destroy()
            ref.destroy()
            P.destroy()
            S.destroy()


@pytest.mark.parametrize("scheme", ["strang", "lie"])
def test_default_graphs_equal_eager_launches(monkeypatch, scheme):
    """Graphs of the default size (about 128 passes of the step body each, repetitions short of
    a whole graph launched directly): 150 and then 70 steps of a batch equal the same batch
    stepped with every pass launched directly (LSX_GRAPH=0), bit for bit."""
    print(f"[case] batch default graphs {scheme}", flush=True)
    monkeypatch.delenv("LSX_GRAPH_PASSES")
    monkeypatch.setenv("LSX_NB", "1")
    monkeypatch.setenv("LSX_KS", "2")
    out = {}
    for graph in ("1", "0"):
        monkeypatch.setenv("LSX_GRAPH", graph)
        made = []
        for k, (spec, W) in enumerate(systems()[:3]):
            S = lsx.System.from_spec(spec)
            P = lsx.Plan(S, 0.004, scheme, 0.5, "mix_fp32")
            st = lsx.State(P, W)
            st.upload(wl.random_state(S.N, W, seed=k))
            made.append((S, P, st))
        B = lsx.Batch([m[2] for m in made])
        B.step(150)
        B.step(70)
        out[graph] = [st.download() for _, _, st in made]
        B.destroy()
        for S, P, st in made:
            st.destroy()
            P.destroy()
            S.destroy()
    for a, b in zip(out["1"], out["0"]):
        assert np.array_equal(a, b)


def test_full_size_batch_members_match_oracle(monkeypatch):
    """The batched workload at full size, in the launch configuration the benchmark times
    (240 chains and 16 twisted bilayers of N up to 4e5, 16 wavepackets each, kappa = 0, Strang,
    mixed FP32, the batch tuner's own shapes and launch mode, graphs by the default rule): three
    chain members (the smallest, the largest and one between) against the oracle's unmerged
    evolution within the derived mixed bound, and every member's mass against its start."""
    print("[case] full-size batch (240 chains + 16 bilayers), mixed FP32", flush=True)
    monkeypatch.delenv("LSX_GRAPH", raising=False)
    monkeypatch.delenv("LSX_GRAPH_PASSES", raising=False)
    specs = wl.batch_specs()
    nsteps, W = 3, 16
    made = []
    try:
        for i, (spec, tau) in enumerate(specs):
            S = lsx.System.from_spec(spec)
            P = lsx.Plan(S, tau, "strang", 0.0, "mix_fp32")
            st = lsx.State(P, W)
            c0 = wl.random_state(S.N, W, seed=i)
            st.upload(c0)
            made.append((S, P, st, c0, spec, tau))
        B = lsx.Batch([m[2] for m in made])
        try:
            B.step(nsteps)
        finally:
            B.destroy()
        Ns = [m[0].N for m in made[:240]]
        picks = sorted({int(np.argmin(Ns)), int(np.argmax(Ns)), int(np.argsort(Ns)[len(Ns) // 2])})
        for i in picks:
            S, P, st, c0, spec, tau = made[i]
            O = splitting.Lifted.from_spec(spec)
            assert np.array_equal(S.index(), O.mn)
            plan = splitting.SplitPlan(O, 0.0)
            oref = plan.evolve(c0, tau, nsteps, "strang")
            bound = mixed_bounds.sequence_bound(plan, mixed_bounds.strang_passes(tau, nsteps, merged=True), "mix_fp32")
            err = colrel(st.download(), oref)
            print(f"  chain {i} N={S.N}: rel err {err:.2e} (bound {bound:.2e})")
            assert err <= bound + 1e-12 * nsteps, (i, S.N, err, bound)
        for i, (S, P, st, c0, spec, tau) in enumerate(made):
            m = st.observables(lsx.OBS_MASS)["mass"]
            m0 = np.sum(np.abs(c0) ** 2, axis=0)
            assert np.abs(m - m0).max() < 1e-6, (i, S.N)
    finally:
        for S, P, st, *_ in made:
            st.destroy()
            P.destroy()
            S.destroy()
