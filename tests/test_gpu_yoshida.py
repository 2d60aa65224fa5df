"""GPU parity of the fourth-order Yoshida composition (triple jump of Strang steps): propagator
slots, trajectories (FP64 per step <= 1e-12 relative L2 against the unmerged oracle), mixed
precision after many steps, and the batched path."""
import numpy as np
import pytest

from oracle import splitting
from paper_2103_14897_amd import lsx
from paper_2103_14897_amd import workloads as wl

pytestmark = pytest.mark.gpu

G1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
G0 = 1.0 - 2.0 * G1


def colrel(a, b):
    return (np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)).max()


def test_yoshida_propagator_slots():
    spec = wl.chain_system(2000.0)
    S = lsx.System.from_spec(spec)
    O = splitting.Lifted.from_spec(spec)
    tau = 0.01
    P = lsx.Plan(S, tau, "yoshida4", 0.0, "fp64")
    try:
        slots = {1: {0: G1 * tau, 1: G1 * tau / 2, 2: (G1 + G0) * tau / 2}, 2: {0: G1 * tau, 2: G0 * tau}}
        for layer, ts in slots.items():
            ptr, rows = S.fibres(layer)
            for slot, t in ts.items():
                for f in (0, len(ptr) // 2, len(ptr) - 2):
                    r = rows[ptr[f]:ptr[f + 1]].astype(np.int64)
                    ref = splitting.propagator_from_hamiltonian(O.fibre_hamiltonian(layer, r, 0.0), t)
                    assert np.abs(P.propagator(layer, slot, f) - ref).max() < 1e-13, (layer, slot, f)
        with pytest.raises(lsx.LsxError):
            P.propagator(2, 1, 0)  # layer 2 has no slot 1 in this scheme
    finally:
        P.destroy()
        S.destroy()


@pytest.mark.parametrize("kappa", [0.0, 0.6])
def test_yoshida_trajectory_tiny(kappa):
    w = wl.tiny_chain()
    S = lsx.System.from_spec(w.spec)
    O = splitting.Lifted.from_spec(w.spec)
    plan = splitting.SplitPlan(O, kappa)
    c = w.initial_state(O.mn)
    P = lsx.Plan(S, w.tau, "yoshida4", kappa, "fp64")
    st = lsx.State(P, 1)
    try:
        st.upload(c)
        st.step(1)
        assert colrel(st.download(), plan.yoshida4_step(c, w.tau)) < 1e-12
        st.upload(c)
        st.step(30)
        ref = plan.evolve(c, w.tau, 30, "yoshida4")
        assert colrel(st.download(), ref) < 30e-12
        m = st.observables(lsx.OBS_MASS)["mass"]
        assert abs(m[0] - 1.0) < 1e-12
    finally:
        st.destroy()
        P.destroy()
        S.destroy()


@pytest.mark.parametrize("which", ["chain", "twisted"])
def test_yoshida_wavepackets(which):
    w = wl.chain(W=16) if which == "chain" else wl.twisted(Ec=1500.0, W=8)
    print(f"[case] yoshida {which}", flush=True)
    S = lsx.System.from_spec(w.spec)
    O = splitting.Lifted.from_spec(w.spec)
    plan = splitting.SplitPlan(O, 0.0)
    c = w.initial_state(O.mn)
    P = lsx.Plan(S, w.tau, "yoshida4", 0.0, "fp64")
    st = lsx.State(P, w.W)
    try:
        st.upload(c)
        st.step(3)
        assert colrel(st.download(), plan.evolve(c, w.tau, 3, "yoshida4")) < 5e-12
        # mixed precision against the FP64 path after 50 steps
        st.upload(c)
        st.step(50)
        ref = st.download()
        for prec in ("mix_fp32", "mix_bf16x3"):
            Pm = lsx.Plan(S, w.tau, "yoshida4", 0.0, prec)
            sm = lsx.State(Pm, w.W)
            sm.upload(c)
            sm.step(50)
            err = colrel(sm.download(), ref)
            print(f"  {prec}: 50 steps rel err vs FP64 {err:.2e}")
            assert err < 1e-6
            sm.destroy()
            Pm.destroy()
    finally:
        st.destroy()
        P.destroy()
        S.destroy()


def test_yoshida_batch_equals_individual(monkeypatch):
    monkeypatch.setenv("LSX_GRAPH", "1")
    monkeypatch.setenv("LSX_GRAPH_PASSES", "2")  # graphs of one body repetition: the second call replays one
    systems = [wl.chain_system(2000.0), wl.chain_system(5000.0, L2=np.sqrt(2.0)), wl.twisted_system(300.0)]
    Ss, Ps, sts, refs = [], [], [], []
    try:
        for k, spec in enumerate(systems):
            S = lsx.System.from_spec(spec)
            P = lsx.Plan(S, 2e-3, "yoshida4", 0.0, "fp64")
            st = lsx.State(P, 4 + k)
            c = wl.random_state(S.N, 4 + k, seed=k)
            st.upload(c)
            ref = lsx.State(P, 4 + k)
            ref.upload(c)
            ref.step(7)
            refs.append(ref)
            Ss.append(S)
            Ps.append(P)
            sts.append(st)
        B = lsx.Batch(sts)
        B.step(3)
        B.step(4)  # second call replays the captured body
        for st, ref in zip(sts, refs):
            assert colrel(st.download(), ref.download()) < 1e-13
        B.destroy()
    finally:
        for o in refs + sts + Ps + Ss:
            o.destroy()
