"""Single-state orbit passes (W = 1, tile shape nb = 8).

Fibres that share one stored propagator (the point-symmetry orbits of the twisted bilayer and
of the chain, the translation classes of the kappa = 1 windows) are multiplied together: a
tile holds row blocks of the shared propagator and the states of up to eight such fibres, so
each propagator chunk is loaded once for the group instead of once per fibre.

* every shape (ks in 1, 2, 4; four-row-block tiles with one row per lane -1, -2, -4, -8) of every precision
  on the chain (groups of two), the twisted bilayer (groups of six and the fixed fibre) and the
  kappa = 1 chain windows (groups of up to eight): single passes of both layers equal the
  per-fibre kernel of the same shape bit for bit (the same products summed in the same order)
  and agree with the oracle's fibre flows (FP64 within 1e-12, the mixed paths within their
  derived bounds, tests/mixed_bounds.py);
* Strang trajectories, whose first pass gathers through the layout tables and whose passes
  apply the kinetic phase (kappa = 0.5) in their epilogue, equal the per-fibre kernel's;
* a plan without shared propagators (LSX_SYMMETRY=0) refuses the shape;
* three layers (the chain trilayer at kappa 0 and 1): every layer's orbit tiles equal the
  per-fibre tiles and agree with the three-layer oracle's fibre flows.
"""
import numpy as np
import pytest

import mixed_bounds
from oracle import splitting
from paper_2103_14897_amd import lsx
from paper_2103_14897_amd import workloads as wl

pytestmark = pytest.mark.gpu

ORBIT_NB = 8


def colrel(a, b):
    return (np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)).max()


def shapes(precision):
    return [1, 2, 4, -1, -2, -4, -8]


def untuned_states(P, n, monkeypatch):
    monkeypatch.setenv("LSX_AUTOTUNE", "0")
    try:
        return [lsx.State(P, 1) for _ in range(n)]
    finally:
        monkeypatch.delenv("LSX_AUTOTUNE")


CASES = [(wl.chain_system(2.0e4), 0.0, 2), (wl.twisted_system(1500.0), 0.0, 6), (wl.chain_system(2.0e4), 1.0, 8)]
IDS = ["chain", "twisted1500", "chain-k1"]


@pytest.mark.parametrize("precision", ["fp64", "mix_fp32", "mix_bf16x3"])
@pytest.mark.parametrize("spec,kappa,gmax", CASES, ids=IDS)
def test_orbit_passes_equal_per_fibre_passes(spec, kappa, gmax, precision, monkeypatch):
    tau = 1e-3
    print(f"[case] orbit passes {spec.name} kappa={kappa} {precision}", flush=True)
    S = lsx.System.from_spec(spec)
    O = splitting.Lifted.from_spec(spec)
    oplan = splitting.SplitPlan(O, kappa)
    P = lsx.Plan(S, tau, "strang", kappa, precision)
    orb, ref = untuned_states(P, 2, monkeypatch)
    try:
        for layer in (1, 2):
            nd, _ = P.sharing(layer)
            assert nd < S.nfibres[layer]
        c = wl.random_state(S.N, 1, seed=11)
        for layer, half, t in ((1, 0, tau), (1, 1, tau / 2), (2, 0, tau)):
            want = oplan.apply_fibres(c, layer, t)
            if precision == "fp64":
                tol = 1e-12
            else:
                tol = mixed_bounds.pass_bound(oplan.propagators(layer, t), precision) + 1e-12
            for ks in shapes(precision):
                orb.set_tuning(layer, ORBIT_NB, ks)
                ref.set_tuning(layer, 1, ks)
                assert orb.tuning(layer)[:2] == (ORBIT_NB, ks)
                orb.upload(c)
                ref.upload(c)
                orb.fibre_pass(layer, half)
                ref.fibre_pass(layer, half)
                got = orb.download()
                assert np.array_equal(got, ref.download()), (layer, half, ks)
                err = colrel(got, want)
                assert err < tol, (layer, half, ks, err, tol)
        print(f"  every shape bitwise equal to the per-fibre kernel; groups up to {gmax}", flush=True)
    finally:
        orb.destroy()
        ref.destroy()
        P.destroy()
        S.destroy()


@pytest.mark.parametrize("precision", ["fp64", "mix_fp32", "mix_bf16x3"])
@pytest.mark.parametrize("which", ["chain", "twisted"])
def test_orbit_trajectories_with_fused_phase(which, precision, monkeypatch):
    spec = wl.chain_system(2.0e4) if which == "chain" else wl.twisted_system(1500.0)
    print(f"[case] orbit trajectories {which} kappa=0.5 {precision}", flush=True)
    S = lsx.System.from_spec(spec)
    P = lsx.Plan(S, 1e-3, "strang", 0.5, precision)
    orb, ref = untuned_states(P, 2, monkeypatch)
    try:
        ks = -2
        for layer in (1, 2):
            orb.set_tuning(layer, ORBIT_NB, ks)
            ref.set_tuning(layer, 1, ks)
        c = wl.random_state(S.N, 1, seed=5)
        orb.upload(c)
        ref.upload(c)
        orb.step(15)
        ref.step(15)
        assert np.array_equal(orb.download(), ref.download())
    finally:
        orb.destroy()
        ref.destroy()
        P.destroy()
        S.destroy()


def test_orbit_shape_needs_shared_propagators(monkeypatch):
    S = lsx.System.from_spec(wl.chain_system(971.0))
    monkeypatch.setenv("LSX_SYMMETRY", "0")
    P = lsx.Plan(S, 1e-3, "strang", 0.0, "fp64")
    monkeypatch.delenv("LSX_SYMMETRY")
    st = untuned_states(P, 1, monkeypatch)[0]
    try:
        assert P.sharing(1)[0] == S.nfibres[1]
        with pytest.raises(lsx.LsxError) as e:
            st.set_tuning(1, ORBIT_NB, 1)
        assert e.value.code == lsx.LSX_E_INVALID
        # the forced shape falls back to per-fibre tiles where nothing is shared
        monkeypatch.setenv("LSX_NB", str(ORBIT_NB))
        monkeypatch.setenv("LSX_KS", "1")
        st2 = lsx.State(P, 1)
        monkeypatch.delenv("LSX_NB")
        monkeypatch.delenv("LSX_KS")
        assert st2.tuning(1)[:2] == (1, 1)
        st2.destroy()
    finally:
        st.destroy()
        P.destroy()
        S.destroy()


@pytest.mark.parametrize("precision", ["fp64", "mix_fp32", "mix_bf16x3"])
@pytest.mark.parametrize("kappa", [0.0, 1.0])
def test_three_layer_orbit_passes(kappa, precision, monkeypatch):
    """Three-layer chain (x -> -x orbits at kappa 0, translation classes at kappa 1): every layer's
    orbit tiles equal the per-fibre tiles of the same shape bit for bit and agree with the
    three-layer oracle's fibre flows."""
    from oracle import multilayer as ml
    spec = wl.chain_layers(2000.0)
    print(f"[case] three-layer orbit passes kappa={kappa} {precision}", flush=True)
    S = lsx.System.layers(spec.d, spec.As, spec.Ec, spec.cutoff, spec.pots)
    O = ml.MultiLifted(spec.d, spec.As, spec.Ec, spec.cutoff, spec.pots)
    oplan = ml.MultiSplitPlan(O, kappa)
    tau = 0.01
    P = lsx.Plan(S, tau, "strang", kappa, precision)
    orb, ref = untuned_states(P, 2, monkeypatch)
    try:
        c = wl.random_state(S.N, 1, seed=13)
        for layer, half, t in ((1, 1, tau / 2), (2, 1, tau / 2), (3, 0, tau)):
            assert P.sharing(layer)[0] < S.nfibres[layer]
            want = oplan.apply_fibres(c, layer, t)
            tol = 1e-12 if precision == "fp64" else 1e-7
            for ks in (2, -4):
                orb.set_tuning(layer, ORBIT_NB, ks)
                ref.set_tuning(layer, 1, ks)
                orb.upload(c)
                ref.upload(c)
                orb.fibre_pass(layer, half)
                ref.fibre_pass(layer, half)
                got = orb.download()
                assert np.array_equal(got, ref.download()), (layer, ks)
                assert colrel(got, want) < tol, (layer, ks)
    finally:
        orb.destroy()
        ref.destroy()
        P.destroy()
        S.destroy()
