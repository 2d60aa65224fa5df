"""GPU parity of the row-split fibre passes (waves on consecutive row blocks sharing an LDS-staged
state operand, each multiplying its own row block's band), forced for every shape against the
oracle: single passes of both layers (the mixed-precision bound, 1e-7 relative L2) and Strang
trajectories against the FP64 path."""
import os

import numpy as np
import pytest

from oracle import splitting
from paper_2103_14897_amd import lsx
from paper_2103_14897_amd import workloads as wl

pytestmark = pytest.mark.gpu


def colrel(a, b):
    return (np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)).max()


SHAPES = [("mix_fp32", nb, ms) for nb, ms in [(1, 2), (1, 4), (2, 2), (2, 4), (2, 8), (4, 2), (4, 4), (4, 8)]] + \
    [("mix_bf16x3", nb, ms) for nb, ms in [(1, 2), (1, 4), (1, 8), (2, 2), (2, 4), (2, 8)]]


@pytest.mark.parametrize("prec,nb,ms", SHAPES)
@pytest.mark.parametrize("which", ["chain", "twisted"])
def test_rowsplit_shapes(prec, nb, ms, which, monkeypatch):
    spec = wl.chain_system(2.0e4) if which == "chain" else wl.twisted_system(1500.0)
    W = 37  # ragged column blocks
    S = lsx.System.from_spec(spec)
    O = splitting.Lifted.from_spec(spec)
    plan = splitting.SplitPlan(O, 0.0)
    tau = 1e-3
    print(f"[case] rowsplit {which} {prec} nb={nb} ms={ms}", flush=True)
    P = lsx.Plan(S, tau, "strang", 0.0, prec)
    P64 = lsx.Plan(S, tau, "strang", 0.0, "fp64")
    monkeypatch.setenv("LSX_NB", str(nb))
    monkeypatch.setenv("LSX_KS", str(-ms))
    st = lsx.State(P, W)
    monkeypatch.delenv("LSX_NB")
    monkeypatch.delenv("LSX_KS")
    ref = lsx.State(P64, W)
    try:
        assert st.tuning(1)[:2] == (nb, -ms) and st.tuning(2)[:2] == (nb, -ms)
        c = wl.random_state(S.N, W, seed=nb + 10 * ms)
        for layer, half, t in ((1, 0, tau), (1, 1, tau / 2), (2, 0, tau)):
            st.upload(c)
            st.fibre_pass(layer, half)
            assert colrel(st.download(), plan.apply_fibres(c, layer, t)) < 1e-7, (layer, half)
        st.upload(c)
        ref.upload(c)
        st.step(20)
        ref.step(20)
        assert colrel(st.download(), ref.download()) < 1e-6
    finally:
        st.destroy()
        ref.destroy()
        P.destroy()
        P64.destroy()
        S.destroy()


@pytest.mark.parametrize("prec", ["fp64", "mix_fp32", "mix_bf16x3"])
@pytest.mark.parametrize("ks", [-1, -2, -4, -8])
@pytest.mark.parametrize("which", ["chain", "twisted"])
def test_single_state_row_lane_tiles(prec, ks, which, monkeypatch):
    """W = 1 tiles of four row blocks with one output row per lane (ks < 0), whose state operand
    is read once per wave: single passes of both layers against the oracle and Strang
    trajectories (kappa 0 and 0.5, the latter with the phase fused into the pass) against the
    one-row-block tiles of the same precision."""
    spec = wl.chain_system(2.0e4) if which == "chain" else wl.twisted_system(1500.0)
    S = lsx.System.from_spec(spec)
    O = splitting.Lifted.from_spec(spec)
    plan = splitting.SplitPlan(O, 0.0)
    tau = 1e-3
    print(f"[case] single-state row-per-lane tiles {which} {prec} ks={ks}", flush=True)
    P = lsx.Plan(S, tau, "strang", 0.0, prec)
    monkeypatch.setenv("LSX_NB", "1")
    monkeypatch.setenv("LSX_KS", str(ks))
    st = lsx.State(P, 1)
    kref = min(-ks, 4)  # the one-row-block tiles take up to four waves
    monkeypatch.setenv("LSX_KS", str(kref))
    ref = lsx.State(P, 1)
    monkeypatch.delenv("LSX_NB")
    monkeypatch.delenv("LSX_KS")
    try:
        assert st.tuning(1)[:2] == (1, ks) and ref.tuning(1)[:2] == (1, kref)
        c = wl.random_state(S.N, 1, seed=-ks)
        tol = 1e-12 if prec == "fp64" else 1e-7
        for layer, half, t in ((1, 0, tau), (1, 1, tau / 2), (2, 0, tau)):
            st.upload(c)
            st.fibre_pass(layer, half)
            assert colrel(st.download(), plan.apply_fibres(c, layer, t)) < tol, (layer, half)
        st.upload(c)
        ref.upload(c)
        st.step(20)
        ref.step(20)
        # the same FP64 products summed in another order (one running sum per row against four
        # per row combined at the end): FP64 rounding of 40 passes over fibres of up to ~400
        assert colrel(st.download(), ref.download()) < 1e-12
    finally:
        st.destroy()
        ref.destroy()
        P.destroy()
    # a kinetic share: the phase fused into the row-per-lane tiles' epilogue
    P = lsx.Plan(S, tau, "strang", 0.5, prec)
    monkeypatch.setenv("LSX_NB", "1")
    monkeypatch.setenv("LSX_KS", str(ks))
    st = lsx.State(P, 1)
    monkeypatch.setenv("LSX_KS", str(kref))
    ref = lsx.State(P, 1)
    monkeypatch.delenv("LSX_NB")
    monkeypatch.delenv("LSX_KS")
    try:
        c = wl.random_state(S.N, 1, seed=7)
        st.upload(c)
        ref.upload(c)
        st.step(20)
        ref.step(20)
        assert colrel(st.download(), ref.download()) < 1e-12
    finally:
        st.destroy()
        ref.destroy()
        P.destroy()
        S.destroy()
