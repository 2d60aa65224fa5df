"""Band-limited fibre products (lsx_plan_band, lsx_plan_fibre_band).

Over one short step an entry P_ab of a fibre propagator arises only through chains of potential
couplings between rows a and b (eq. 3.6), each link of order t|v|, so the entries fall off fast
away from the diagonal.  For every block of 16 propagator rows the plan records the range of
column chunks holding an entry with |Re| + |Im| >= tol, and the passes multiply only those.

* the recorded bands against the oracle's propagators (eigh, FP64), for every slot the plan
  holds: every chunk whose largest entry reaches 2 tol lies inside the band, and the band's
  first and last chunks reach tol / 2, so the band is also tight;
* banded trajectories against dense ones (band_tol < 0): FP64 within the left-out entries'
  bound (Lmax tol per pass) plus rounding, the mixed paths within the sum of both runs' derived
  bounds (tests/mixed_bounds.py); the oracle
  comparisons of every other GPU test run on the default, banded plans;
* the bands of the default tolerances leave out most of the products on the 1D chain (the
  BF16x3 format's 32-column chunks less so on its short layer-1 fibres).
"""
import numpy as np
import pytest

import mixed_bounds
from oracle import splitting
from paper_2103_14897_amd import lsx
from paper_2103_14897_amd import workloads as wl

pytestmark = pytest.mark.gpu

ASYM1 = {(1,): 0.6 + 0.45j, (-1,): 0.6 - 0.45j, (2,): 0.2 - 0.1j, (-2,): 0.2 + 0.1j}
ASYM2 = {(1,): 0.5 - 0.3j, (-1,): 0.5 + 0.3j, (0,): 0.15}


def colrel(a, b):
    return (np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)).max()


def chunk_max(P, mixed, cw):
    """Largest |Re| + |Im| of every (16-row block, cw-column chunk) of the zero-padded P (of its
    off-diagonal part E for the mixed formats)."""
    L = P.shape[0]
    M = np.abs(P.real) + np.abs(P.imag)
    if mixed:
        M[np.arange(L), np.arange(L)] = 0.0
    Lp = -(-L // max(16, cw)) * max(16, cw)
    Z = np.zeros((Lp, Lp))
    Z[:L, :L] = M
    return Z.reshape(Lp // 16, 16, Lp // cw, cw).max(axis=(1, 3))[: (L + 15) // 16]


CASES = [
    (wl.chain_system(2.0e4), 1e-3, 0.0),
    (wl.chain_system(971.0, pot1=ASYM1, pot2=ASYM2), 0.01, 0.5),
    (wl.twisted_system(1500.0), 5e-3, 0.0),
    (wl.chain_system(2.0e4), 1e-3, 1.0),
]
IDS = ["chain", "complex-k05", "twisted1500", "chain-k1"]


@pytest.mark.parametrize("precision", ["fp64", "mix_fp32", "mix_bf16x3"])
@pytest.mark.parametrize("spec,tau,kappa", CASES, ids=IDS)
def test_bands_cover_the_oracle_propagators(spec, tau, kappa, precision, monkeypatch):
    tol = 1e-9  # well above the rounding noise of the propagators' far entries
    cw = 32 if precision == "mix_bf16x3" else 4
    print(f"[case] band {spec.name} tau={tau} kappa={kappa} {precision}", flush=True)
    monkeypatch.setenv("LSX_SYMMETRY", "0")  # plan rows in ascending order, as the oracle's
    S = lsx.System.from_spec(spec)
    P = lsx.Plan(S, tau, "strang", kappa, precision, band_tol=tol)
    monkeypatch.delenv("LSX_SYMMETRY")
    O = splitting.Lifted.from_spec(spec)
    plan = splitting.SplitPlan(O, kappa)
    try:
        assert P.band(1)[0] == tol
        for layer, times in ((1, (tau, tau / 2)), (2, (tau,))):
            props = [plan.propagators(layer, t) for t in times]
            for f in range(S.nfibres[layer]):
                m = np.maximum.reduce([chunk_max(pp[f], precision != "fp64", cw) for pp in props])
                band = P.fibre_band(layer, f)
                assert band.shape[0] == m.shape[0]
                for rb in range(m.shape[0]):
                    lo, hi = band[rb] // cw
                    assert band[rb, 0] % cw == 0 and band[rb, 1] % cw == 0 and 0 <= lo < hi <= m.shape[1]
                    big = np.nonzero(m[rb] >= 2 * tol)[0]
                    if len(big):
                        assert lo <= big[0] and big[-1] < hi, (layer, f, rb, band[rb], big)
                        assert m[rb, lo] >= tol / 2 and m[rb, hi - 1] >= tol / 2, (layer, f, rb)
                    elif not np.any(m[rb] >= tol / 2):
                        assert hi - lo == 1, (layer, f, rb)
    finally:
        P.destroy()
        S.destroy()


@pytest.mark.parametrize("precision", ["fp64", "mix_fp32", "mix_bf16x3"])
@pytest.mark.parametrize("which", ["chain", "twisted"])
def test_banded_steps_equal_dense_steps(which, precision):
    w = wl.chain(W=64) if which == "chain" else wl.twisted(Ec=1500.0, W=16)
    nsteps = 50 if which == "chain" else 20
    print(f"[case] banded vs dense {which} {precision} {nsteps} steps", flush=True)
    S = lsx.System.from_spec(w.spec)
    O = splitting.Lifted.from_spec(w.spec)
    c0 = w.initial_state(O.mn)
    Pb = lsx.Plan(S, w.tau, "strang", 0.0, precision)
    Pd = lsx.Plan(S, w.tau, "strang", 0.0, precision, band_tol=-1.0)
    sb, sd = lsx.State(Pb, w.W), lsx.State(Pd, w.W)
    try:
        assert Pd.band(1)[0] == 0.0 and Pd.band(1)[1] == Pd.band(1)[2]
        tol = 2.0 ** -53 if precision == "fp64" else 2.0 ** -44
        assert Pb.band(1)[0] == tol
        sb.upload(c0)
        sd.upload(c0)
        sb.step(nsteps)
        sd.step(nsteps)
        err = colrel(sb.download(), sd.download())
        if precision == "fp64":
            # left-out entries: at most Lmax tol per pass; the rest is rounding order
            Lmax = max(len(r) for l in (1, 2) for _, r in O.fib[l])
            bound = 2 * nsteps * Lmax * tol + 1e-13
        else:
            oplan = splitting.SplitPlan(O, 0.0)
            passes = mixed_bounds.strang_passes(w.tau, nsteps)
            bound = (mixed_bounds.sequence_bound(oplan, passes, precision)
                     + sum(mixed_bounds.pass_bound(oplan.propagators(l, t), precision, band_tol=0.0)
                           for l, t in passes))
        print(f"  banded vs dense {err:.2e} (bound {bound:.2e})", flush=True)
        assert err <= bound
    finally:
        for o in (sb, sd, Pb, Pd, S):
            o.destroy()


@pytest.mark.parametrize("precision", ["fp64", "mix_fp32", "mix_bf16x3"])
def test_default_bands_skip_most_chain_products(precision):
    w = wl.chain(W=64)
    S = lsx.System.from_spec(w.spec)
    P = lsx.Plan(S, w.tau, "strang", 0.0, precision)
    try:
        for layer in (1, 2):
            tol, kept, dense, skept, srows = P.band(layer, stored=True)
            print(f"[case] chain band {precision} layer {layer}: tol {tol:.1e}, kept {kept / dense:.3f}, "
                  f"stored {skept / kept:.3f} of it ({P.sharing(layer)[0]} of {S.nfibres[layer]} fibres)", flush=True)
            # x -> -x maps the chain onto itself, so mirror fibres share one stored propagator
            assert 0 < skept < kept and 0 < srows < S.N
            # BF16x3 chunks are 32 columns wide, coarse against the chain's short layer-1 fibres
            assert 0 < kept < (0.9 if precision == "mix_bf16x3" and layer == 1 else 0.7) * dense
    finally:
        P.destroy()
        S.destroy()
