"""Batched uneven systems: one grouped launch per pass over several systems.

Each system stepped inside a batch must equal the same system stepped on its own (up to
the summation order of a different tile shape), for every scheme and precision, with
systems of different lattices, cutoffs, dimensions and wavepacket counts; the replayed
HIP graph of the step body must give the same result on every call.
"""
import math

import numpy as np
import pytest

from paper_2103_14897_amd import lsx
from paper_2103_14897_amd import workloads as wl

pytestmark = pytest.mark.gpu


def colrel(a, b):
    return (np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)).max()


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
    made = []
    for spec, W in systems():
        S = lsx.System.from_spec(spec)
        P = lsx.Plan(S, 0.004, scheme, kappa, precision)
        c0 = wl.random_state(S.N, W, seed=W)
        ref_st = lsx.State(P, W)
        ref_st.upload(c0)
        ref_st.step(7)
        ref = ref_st.download()
        ref_st.destroy()
        st = lsx.State(P, W)
        st.upload(c0)
        made.append((S, P, st, c0, ref))
    B = lsx.Batch([m[2] for m in made])
    B.step(7)
    # two runs of a mixed path that differ only in the FP32 summation order of their tiles:
    # each run's own rounding is <= ~1.3e-10 relative per pass against FP64, so after
    # 7 steps (14 passes) the two differ by well under 1e-8
    tol = 1e-13 if precision == "fp64" else 1e-8
    for S, P, st, c0, ref in made:
        assert colrel(st.download(), ref) < tol
    # a second call replays the captured body graph from a fresh upload
    for S, P, st, c0, ref in made:
        st.upload(c0)
    B.step(7)
    for S, P, st, c0, ref in made:
        assert colrel(st.download(), ref) < tol
    B.destroy()
    for S, P, st, c0, ref in made:
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
    stepped on its own.  Three-layer Lie has an odd number of passes per step, so its graph
    holds two repetitions and an odd leftover runs eagerly (7 steps: head, 2 replays, 1 extra,
    tail)."""
    print(f"[case] three-layer batch {scheme}", flush=True)
    specs = [(wl.chain_layers(800.0), 8), (wl.chain_layers(1500.0, periods=(1.0, math.sqrt(2.0), math.sqrt(3.0))), 5),
             (wl.twisted_layers(120.0), 4)]
    made = []
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
            made.append((S, P, st, ref, c0))
        B = lsx.Batch([m[2] for m in made])
        for _ in range(2):  # the second call replays the captured graph
            for S, P, st, ref, c0 in made:
                st.upload(c0)
            B.step(7)
            for S, P, st, ref, c0 in made:
                assert colrel(st.download(), ref.download()) < 1e-13
        B.destroy()
    finally:
        for S, P, st, ref, c0 in made:
            st.destroy()
            ref.destroy()
            P.destroy()
            S.destroy()


def test_example3_batch_and_mixed_layer_counts():
    made = []
    try:
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
        B = lsx.Batch([m[2] for m in made])
        B.step(6)
        for S, P, st, ref in made:
            assert colrel(st.download(), ref.download()) < 1e-8
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
