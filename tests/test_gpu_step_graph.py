"""Captured step graphs of lsx_step.

A call that repeats the step body often enough replays HIP graphs of many body repetitions
instead of launching every pass from the host: graphs of about 512 passes (LSX_GRAPH_PASSES)
for the bulk of the call, then halved sizes down to about 32 passes (LSX_GRAPH_MIN_PASSES) for
its remainder.  The graphs are kept with the state, one per size and arrangement of its two
arrays (an owned state's arrays swap roles after a call with an odd number of passes), up to
16 of them (the least recently used is replaced), and rebuilt after the tile shape or the
store mode changes.  The launches are the same, so the results must be bit-identical to
launching every pass directly (LSX_GRAPH=0):

* every scheme (three-layer Lie has an odd body), kappa 0 and 0.5 (phase sub-steps inside the
  body), FP64 and mixed FP32, over a sequence of calls of different lengths: shorter than one
  graph, several graphs with a remainder, odd and even pass counts;
* ladders of graph sizes down to one or two body repetitions, every scheme, over calls whose
  remainders take different sizes;
* the default sizes over long calls, an owned state and a wrapped state;
* more graphs than the state keeps (sizes changed between calls), so that graphs are replaced;
* the configuration the benchmark times (the Ec = 2e4 chain, 64 wavepackets, tuned shapes,
  2000 steps in one call), FP64 and mixed FP32;
* a changed tile shape and store mode between calls;
* a caller's own stream capture of lsx_step (the library then launches every pass into it):
  one replay equals direct stepping.
"""
import numpy as np
import pytest
import torch

from paper_2103_14897_amd import lsx
from paper_2103_14897_amd import workloads as wl

pytestmark = pytest.mark.gpu

CALLS = [1, 9, 2, 30, 5, 17]


def run(monkeypatch, make, scheme, kappa, precision, W, calls, graph, passes=None, change=None, wrap=False,
        min_passes=None, sizes=None):
    monkeypatch.setenv("LSX_GRAPH", graph)
    if passes is None:
        monkeypatch.delenv("LSX_GRAPH_PASSES", raising=False)
    else:
        monkeypatch.setenv("LSX_GRAPH_PASSES", str(passes))
    if min_passes is None:
        monkeypatch.delenv("LSX_GRAPH_MIN_PASSES", raising=False)
    else:
        monkeypatch.setenv("LSX_GRAPH_MIN_PASSES", str(min_passes))
    monkeypatch.setenv("LSX_NB", "1")
    monkeypatch.setenv("LSX_KS", "2")
    S = make()
    P = lsx.Plan(S, 2e-3, scheme, kappa, precision)
    t = None
    if wrap:
        t = torch.zeros((S.N, W), dtype=torch.complex128, device="cuda")
        st = lsx.State(P, W, dev_ptr=t.data_ptr())
    else:
        st = lsx.State(P, W)
    monkeypatch.delenv("LSX_NB")
    monkeypatch.delenv("LSX_KS")
    try:
        st.upload(wl.random_state(S.N, W, seed=3))
        for i, n in enumerate(calls):
            if change is not None and i == 2:
                change(st)
            if sizes is not None:
                monkeypatch.setenv("LSX_GRAPH_PASSES", str(sizes[i % len(sizes)]))
            st.step(n)
        return st.download()
    finally:
        st.destroy()
        P.destroy()
        S.destroy()


def two_layer():
    return lsx.System.from_spec(wl.chain_system(2000.0))


def three_layer():
    spec = wl.chain_layers(600.0)
    return lsx.System.layers(spec.d, spec.As, spec.Ec, spec.cutoff, spec.pots)


@pytest.mark.parametrize("precision", ["fp64", "mix_fp32"])
@pytest.mark.parametrize("kappa", [0.0, 0.5])
@pytest.mark.parametrize("scheme", ["strang", "lie", "yoshida4", "strang_cn", "lie_be"])
def test_small_graphs_equal_direct_launches(monkeypatch, scheme, kappa, precision):
    print(f"[case] step graphs {scheme} kappa={kappa} {precision}", flush=True)
    a = run(monkeypatch, two_layer, scheme, kappa, precision, 8, CALLS, "1", passes=4)
    b = run(monkeypatch, two_layer, scheme, kappa, precision, 8, CALLS, "0")
    assert np.array_equal(a, b)


@pytest.mark.parametrize("scheme", ["lie", "strang"])
def test_three_layer_graphs_equal_direct_launches(monkeypatch, scheme):
    print(f"[case] step graphs three layers {scheme}", flush=True)
    a = run(monkeypatch, three_layer, scheme, 0.0, "fp64", 4, CALLS, "1", passes=3)
    b = run(monkeypatch, three_layer, scheme, 0.0, "fp64", 4, CALLS, "0")
    assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", ["fp64", "mix_fp32"])
@pytest.mark.parametrize("scheme", ["strang", "lie", "yoshida4", "strang_cn", "lie_be"])
def test_graph_ladder_equals_direct_launches(monkeypatch, scheme, precision):
    print(f"[case] step graph ladder {scheme} {precision}", flush=True)
    calls = [40, 3, 23, 17, 9, 64]
    a = run(monkeypatch, two_layer, scheme, 0.5, precision, 8, calls, "1", passes=32, min_passes=2)
    b = run(monkeypatch, two_layer, scheme, 0.5, precision, 8, calls, "0")
    assert np.array_equal(a, b)


@pytest.mark.parametrize("scheme", ["lie", "strang"])
def test_three_layer_graph_ladder_equals_direct_launches(monkeypatch, scheme):
    print(f"[case] step graph ladder three layers {scheme}", flush=True)
    calls = [30, 7, 19, 12]
    a = run(monkeypatch, three_layer, scheme, 0.0, "fp64", 4, calls, "1", passes=24, min_passes=3)
    b = run(monkeypatch, three_layer, scheme, 0.0, "fp64", 4, calls, "0")
    assert np.array_equal(a, b)


def test_graph_cache_replacement(monkeypatch):
    """Twenty graph sizes over forty calls (both arrangements of the arrays): more graphs than the
    state keeps, so the least recently used ones are replaced and rebuilt."""
    print("[case] step graph cache replacement", flush=True)
    calls = [25, 26] * 20
    sizes = [2 * (i // 2 + 1) for i in range(40)]
    a = run(monkeypatch, two_layer, "strang", 0.0, "mix_fp32", 8, calls, "1", min_passes=2, sizes=sizes)
    b = run(monkeypatch, two_layer, "strang", 0.0, "mix_fp32", 8, calls, "0")
    assert np.array_equal(a, b)


@pytest.mark.parametrize("wrap", [False, True])
def test_default_graphs_equal_direct_launches(monkeypatch, wrap):
    print(f"[case] step graphs default size wrap={wrap}", flush=True)
    calls = [150, 70, 201, 64]
    a = run(monkeypatch, two_layer, "strang", 0.0, "mix_fp32", 16, calls, "1", wrap=wrap)
    b = run(monkeypatch, two_layer, "strang", 0.0, "mix_fp32", 16, calls, "0", wrap=wrap)
    assert np.array_equal(a, b)


def test_graphs_follow_tuning_changes(monkeypatch):
    print("[case] step graphs after set_tuning / set_store_mode", flush=True)

    def change(st):
        st.set_tuning(1, 1, 4)
        st.set_tuning(2, 2, 1)
        st.set_store_mode(1)

    a = run(monkeypatch, two_layer, "strang", 0.0, "fp64", 24, CALLS, "1", passes=4, change=change)
    b = run(monkeypatch, two_layer, "strang", 0.0, "fp64", 24, CALLS, "0", change=change)
    assert np.array_equal(a, b)


def test_caller_capture_of_step(monkeypatch):
    """lsx_step inside the caller's own capture launches every pass into it; one replay of the
    caller's graph equals stepping directly."""
    print("[case] step inside a caller's stream capture", flush=True)
    monkeypatch.setenv("LSX_NB", "1")
    monkeypatch.setenv("LSX_KS", "2")
    S = two_layer()
    P = lsx.Plan(S, 2e-3, "strang", 0.5, "mix_fp32")
    st, ref = lsx.State(P, 8), lsx.State(P, 8)
    try:
        c = wl.random_state(S.N, 8, seed=4)
        st.upload(c)
        ref.upload(c)
        s = torch.cuda.Stream()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            st.step(300, s)
        g.replay()
        torch.cuda.synchronize()
        monkeypatch.setenv("LSX_GRAPH", "0")
        ref.step(300)
        assert np.array_equal(st.download(), ref.download())
        del g
    finally:
        st.destroy()
        ref.destroy()
        P.destroy()
        S.destroy()


@pytest.mark.parametrize("precision", ["fp64", "mix_fp32"])
def test_headline_chain_graphs_equal_direct_launches(monkeypatch, precision):
    """The configuration the benchmark times: the Ec = 2e4 chain (N = 5149), 64 wavepackets,
    Strang tau = 1e-3, the tuner's own tile shapes and store mode, 2000 steps in one call
    (graph ladder from the default sizes) against the same state stepped with every pass
    launched directly."""
    print(f"[case] headline chain, 2000 steps, graphs vs direct, {precision}", flush=True)
    monkeypatch.delenv("LSX_GRAPH_PASSES", raising=False)
    monkeypatch.delenv("LSX_GRAPH_MIN_PASSES", raising=False)
    monkeypatch.delenv("LSX_GRAPH", raising=False)
    w = wl.chain(2.0e4, 64)
    S = lsx.System.from_spec(w.spec)
    P = lsx.Plan(S, w.tau, "strang", 0.0, precision)
    st = lsx.State(P, 64)
    try:
        c0 = w.initial_state(S.index())
        out = {}
        for graph in ("1", "0"):
            monkeypatch.setenv("LSX_GRAPH", graph)
            st.upload(c0)
            st.step(2000)
            out[graph] = st.download()
        assert np.array_equal(out["1"], out["0"])
        assert np.isfinite(out["1"]).all()
    finally:
        st.destroy()
        P.destroy()
        S.destroy()
