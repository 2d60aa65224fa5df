"""GPU tests of the boundary's auxiliary behaviour through the C-ABI: the descriptor-form calls,
pinned tile shapes and store modes (bitwise-repeatable runs), checkpoint and resume of the
two-layer FP64 path, non-finite observables, and the unwinding of failed set-ups (allocation
and eigensolver failures injected from the host)."""
import numpy as np
import pytest

from oracle import splitting
from paper_2103_14897_amd import lsx
from paper_2103_14897_amd import workloads as wl

pytestmark = pytest.mark.gpu


def colrel(a, b):
    return (np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)).max()


def pin_like(dst, src, nlayers=2):
    """Give state `dst` the tile shapes, prefetch depths and store mode `src` was tuned to."""
    for layer in range(1, nlayers + 1):
        nb, ks, _ = src.tuning(layer)
        dst.set_tuning(layer, nb, ks, src.prefetch(layer))
    dst.set_store_mode(src.store_mode()[0])


def test_descriptor_plan_max_wavepackets_and_wrap():
    import torch

    w = wl.chain(Ec=971.0, W=8)
    print("[case] descriptor plan, chain Ec=971 W=8", flush=True)
    spec = w.spec
    S = lsx.System.from_desc(spec.d, spec.A1, spec.A2, spec.Ec, spec.cutoff, spec.pot1, spec.pot2)
    P = lsx.Plan(S, w.tau, "strang", 0.0, "fp64", max_wavepackets=8)
    try:
        with pytest.raises(lsx.LsxError) as e:
            lsx.State(P, 9)
        assert e.value.code == lsx.LSX_E_INVALID
        O = splitting.Lifted.from_spec(spec)
        c0 = w.initial_state(O.mn)
        own = lsx.State(P, 8)
        own.upload(c0)
        own.step(5)
        t = torch.from_numpy(c0).to("cuda")
        torch.cuda.synchronize()
        wrapped = lsx.State(P, 8, dev_ptr=t.data_ptr())  # lsx_state_wrap
        pin_like(wrapped, own)
        wrapped.step(5)
        torch.cuda.synchronize()
        got = t.cpu().numpy()
        assert colrel(got, splitting.SplitPlan(O, 0.0).evolve(c0, w.tau, 5)) < 5e-12
        # same plan, same pinned shapes: the owned and the wrapped state agree bit for bit
        assert np.array_equal(got, own.download())
        wrapped.destroy()
        own.destroy()
    finally:
        P.destroy()
        S.destroy()


@pytest.mark.parametrize("precision", ["fp64", "mix_fp32", "mix_bf16x3"])
def test_pinned_tuning_gives_bitwise_repeatable_steps(precision):
    """Two states whose tile shapes and store modes are pinned to the same values step bit
    for bit alike; a shape the kernels are not built for is refused and changes nothing."""
    w = wl.chain(Ec=2.0e4, W=64)
    print(f"[case] pinned tuning chain Ec=2e4 W=64 {precision}", flush=True)
    S = lsx.System.from_spec(w.spec)
    P = lsx.Plan(S, w.tau, "strang", 0.0, precision)
    a, b = lsx.State(P, 64), lsx.State(P, 64)
    try:
        c0 = wl.random_state(S.N, 64, seed=3)
        # pin both to a shape other than the tuned one for layer 1, and to a's choice for layer 2
        nb, ks, _ = a.tuning(1)
        alt = (2, 2) if (nb, ks) != (2, 2) else (1, 4)
        for st in (a, b):
            st.set_tuning(1, alt[0], alt[1], 0)
        nb2, ks2, _ = a.tuning(2)
        b.set_tuning(2, nb2, ks2, a.prefetch(2))
        b.set_store_mode(a.store_mode()[0])
        assert b.tuning(1)[:2] == alt and b.tuning(1)[2] == 0.0
        with pytest.raises(lsx.LsxError) as e:
            b.set_tuning(1, 3, 2, 0)
        assert e.value.code == lsx.LSX_E_INVALID
        with pytest.raises(lsx.LsxError):
            b.set_tuning(1, 1, -2 if precision == "fp64" else 3, 0)
        with pytest.raises(lsx.LsxError):
            b.set_store_mode(2)
        assert b.tuning(1)[:2] == alt
        for st in (a, b):
            st.upload(c0)
            st.step(20)
        assert np.array_equal(a.download(), b.download())
    finally:
        for o in (a, b, P, S):
            o.destroy()


@pytest.mark.parametrize("kappa", [0.0, 1.0])
def test_checkpoint_resume_is_bitwise(kappa):
    """A state is (plan, coefficients): K1 steps, download, a new state with the same pinned
    shapes, upload, K2 steps gives bit for bit what K1 then K2 steps in two calls on one state
    give (half steps are never merged across calls); both agree with the oracle's K1 + K2
    unmerged steps to the FP64 bar."""
    w = wl.chain(Ec=2.0e4, W=16)
    print(f"[case] resume chain Ec=2e4 W=16 kappa={kappa}", flush=True)
    S = lsx.System.from_spec(w.spec)
    P = lsx.Plan(S, w.tau, "strang", kappa, "fp64")
    O = splitting.Lifted.from_spec(w.spec)
    c0 = w.initial_state(O.mn)
    K1, K2 = 7, 5
    a = lsx.State(P, 16)
    try:
        a.upload(c0)
        a.step(K1)
        a.step(K2)
        ref = a.download()
        b = lsx.State(P, 16)
        pin_like(b, a)
        b.upload(c0)
        b.step(K1)
        ck = b.download()
        b.destroy()
        c = lsx.State(P, 16)
        pin_like(c, a)
        c.upload(ck)
        c.step(K2)
        got = c.download()
        c.destroy()
        assert np.array_equal(got, ref)
        oref = splitting.SplitPlan(O, kappa).evolve(c0, w.tau, K1 + K2)
        assert colrel(got, oref) < 1e-12 * (K1 + K2)
    finally:
        a.destroy()
        P.destroy()
        S.destroy()


def test_nonfinite_state_reports_nonfinite_observables():
    w = wl.chain(Ec=971.0, W=4)
    print("[case] non-finite observables", flush=True)
    S = lsx.System.from_spec(w.spec)
    P = lsx.Plan(S, w.tau, "strang", 0.0, "fp64")
    st = lsx.State(P, 4)
    try:
        c = wl.random_state(S.N, 4, seed=1)
        st.upload(c)
        m = st.observables(lsx.OBS_MASS | lsx.OBS_ENERGY)
        assert np.all(np.isfinite(m["mass"])) and np.all(np.isfinite(m["energy"]))
        for bad in (np.nan, np.inf):
            c2 = c.copy()
            c2[S.N // 2, 2] = bad
            st.upload(c2)
            for mask in (lsx.OBS_MASS, lsx.OBS_ENERGY, lsx.OBS_FIBRE_MASS_1):
                with pytest.raises(lsx.LsxError) as e:
                    st.observables(mask)
                assert e.value.code == lsx.LSX_E_NONFINITE
        # a finite state afterwards is fine again
        st.upload(c)
        assert np.allclose(st.observables(lsx.OBS_MASS)["mass"], m["mass"], rtol=0, atol=0)
    finally:
        for o in (st, P, S):
            o.destroy()


def test_injected_failures_unwind(monkeypatch):
    """Every device allocation of plan and state creation is made to fail in turn
    (LSX_TEST_FAIL_ALLOC=k): each attempt reports LSX_E_OOM and leaves the library holding
    exactly the buffers it held before; an injected eigensolver failure reports LSX_E_EIG the
    same way; afterwards the same set-up succeeds."""
    w = wl.chain(Ec=971.0, W=16)
    print("[case] failure injection", flush=True)
    S = lsx.System.from_spec(w.spec)
    try:
        base = lsx.live_buffers()
        for precision in ("fp64", "mix_bf16x3"):
            k = 1
            while True:
                assert k < 400, "allocation count did not converge"
                monkeypatch.setenv("LSX_TEST_FAIL_ALLOC", str(k))
                try:
                    P = lsx.Plan(S, w.tau, "strang", 0.0, precision)
                except lsx.LsxError as e:
                    assert e.code == lsx.LSX_E_OOM, (k, e)
                    assert lsx.live_buffers() == base, k
                    k += 1
                    continue
                monkeypatch.delenv("LSX_TEST_FAIL_ALLOC")
                break
            # the plan made it: now fail the state's allocations in turn
            pbase = lsx.live_buffers()
            j = 1
            while True:
                assert j < 400
                monkeypatch.setenv("LSX_TEST_FAIL_ALLOC", str(j))
                try:
                    st = lsx.State(P, 16)
                except lsx.LsxError as e:
                    assert e.code == lsx.LSX_E_OOM, (j, e)
                    assert lsx.live_buffers() == pbase, j
                    j += 1
                    continue
                monkeypatch.delenv("LSX_TEST_FAIL_ALLOC")
                break
            print(f"  {precision}: {k - 1} plan and {j - 1} state allocations failed in turn and unwound")
            assert k > 5 and j > 2
            c0 = wl.random_state(S.N, 16, seed=4)
            st.upload(c0)
            st.step(3)
            assert np.all(np.isfinite(st.download()))
            st.destroy()
            P.destroy()
            assert lsx.live_buffers() == base
        monkeypatch.setenv("LSX_TEST_FAIL_EIG", "1")
        with pytest.raises(lsx.LsxError) as e:
            lsx.Plan(S, w.tau, "strang", 0.0, "fp64")
        assert e.value.code == lsx.LSX_E_EIG
        assert lsx.live_buffers() == base
        monkeypatch.delenv("LSX_TEST_FAIL_EIG")
        P = lsx.Plan(S, w.tau, "strang", 0.0, "fp64")
        P.destroy()
        assert lsx.live_buffers() == base
    finally:
        S.destroy()
