"""Pass output store modes and the reported prefetch depth.  Ordinary and non-temporal stores
give bit-identical trajectories (the mode only changes where the written lines live, never a
value) on two-layer, three-layer and shared-block systems in every precision; the tuner
reports a store mode with both cycle times measured, and the prefetch depth it chose."""
import numpy as np
import pytest

from paper_2103_14897_amd import lsx
from paper_2103_14897_amd import workloads as wl

pytestmark = pytest.mark.gpu


def systems():
    yield "chain", lsx.System.from_spec(wl.chain_system(2000.0))
    yield "twisted", lsx.System.from_spec(wl.twisted_system(300.0))
    spec = wl.twisted_layers(60.0)
    yield "trilayer", lsx.System.layers(spec.d, spec.As, spec.Ec, spec.cutoff, spec.pots)
    spec = wl.example3_system(200.0)
    yield "example3", lsx.System.blocks(spec.Rs, spec.groups, spec.Ec, spec.layers, spec.pots)


@pytest.mark.parametrize("precision,nb,ks", [("fp64", 1, 2), ("fp64", 2, 1), ("mix_fp32", 1, 4),
                                             ("mix_fp32", 2, -4), ("mix_bf16x3", 1, 2), ("mix_bf16x3", 2, -2)])
def test_store_modes_bit_identical(monkeypatch, precision, nb, ks):
    # one forced tile shape, so that both states sum in the same order
    monkeypatch.setenv("LSX_NB", str(nb))
    monkeypatch.setenv("LSX_KS", str(ks))
    W = 24
    for name, S in systems():
        print(f"[case] store modes {name} N={S.N} {precision} nb={nb} ks={ks}", flush=True)
        P = None
        try:
            P = lsx.Plan(S, 5e-3, "strang", 0.0, precision)
            c = wl.random_state(S.N, W, seed=5)
            out = []
            for nt in (0, 1):
                monkeypatch.setenv("LSX_NT", str(nt))
                st = lsx.State(P, W)
                try:
                    assert st.store_mode()[0] == nt
                    assert st.tuning(1)[:2] == (nb, ks)
                    st.upload(c)
                    st.step(7)
                    out.append(st.download())
                finally:
                    st.destroy()
            assert np.array_equal(out[0], out[1]), name
        finally:
            if P is not None:
                P.destroy()
            S.destroy()


def test_store_mode_is_tuned():
    S = lsx.System.from_spec(wl.chain_system(2.0e4))
    P = lsx.Plan(S, 1e-3, "strang", 0.0, "mix_fp32")
    try:
        st = lsx.State(P, 64)
        nt, us = st.store_mode()
        print(f"  chain Ec=2e4 W=64: mode {nt}, cycle us {us}")
        assert nt in (0, 1) and us[0] > 0.0 and us[1] > 0.0
        assert nt == (1 if us[1] < us[0] else 0)
        st.destroy()
        st1 = lsx.State(P, 1)  # matrix-vector passes keep ordinary stores, untimed
        assert st1.store_mode() == (0, (0.0, 0.0))
        st1.destroy()
    finally:
        P.destroy()
        S.destroy()


def test_prefetch_depth_reported(monkeypatch):
    """The tile tuner's prefetch depth: 1 or 2 on the K-split shapes of the FP64 and mixed FP32
    paths, 0 (library default) for row-split shapes, BF16x3, forced shapes and LSX_PREFETCH."""
    S = lsx.System.from_spec(wl.chain_system(2.0e4))
    try:
        for precision in ("fp64", "mix_fp32", "mix_bf16x3"):
            P = lsx.Plan(S, 1e-3, "strang", 0.0, precision)
            try:
                st = lsx.State(P, 64)
                for layer in (1, 2):
                    u, ks = st.prefetch(layer), st.tuning(layer)[1]
                    print(f"  {precision} layer {layer}: ks {ks} prefetch {u}")
                    if precision != "mix_bf16x3" and ks > 0:
                        assert u in (1, 2)
                    else:
                        assert u == 0
                st.destroy()
                for env in (("LSX_NB", "1"), ("LSX_PREFETCH", "1")):
                    monkeypatch.setenv(*env)
                    st = lsx.State(P, 64)
                    assert st.prefetch(1) == 0 and st.prefetch(2) == 0, env
                    st.destroy()
                    monkeypatch.delenv(env[0])
            finally:
                P.destroy()
    finally:
        S.destroy()


def test_autotune_off_keeps_defaults(monkeypatch):
    """LSX_AUTOTUNE=0: nothing is timed at creation; default shape, library-default depth and
    ordinary stores, and the step still matches a tuned state to FP64 rounding (the tuned shape
    may sum in another order)."""
    S = lsx.System.from_spec(wl.chain_system(2000.0))
    P = lsx.Plan(S, 1e-3, "strang", 0.0, "fp64")
    try:
        c = wl.random_state(S.N, 16, seed=2)
        st = lsx.State(P, 16)
        st.upload(c)
        st.step(20)
        ref = st.download()
        st.destroy()
        monkeypatch.setenv("LSX_AUTOTUNE", "0")
        st = lsx.State(P, 16)
        try:
            assert st.store_mode() == (0, (0.0, 0.0))
            for layer in (1, 2):
                assert st.tuning(layer) == (1, 2, 0.0) and st.prefetch(layer) == 0
            st.upload(c)
            st.step(20)
            out = st.download()
            err = (np.linalg.norm(out - ref, axis=0) / np.linalg.norm(ref, axis=0)).max()
            assert err < 1e-12, err
        finally:
            st.destroy()
    finally:
        P.destroy()
        S.destroy()
