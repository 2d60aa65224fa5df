"""The batched FP64 eigensolver behind every fibre propagator (P(t) = U f(Lambda) U^H, Sec. 4.2
exact sub-flows, Alg. 2 / eq. 4.6 rational factors): fibres longer than 96 rows (after the
real embedding of complex Hamiltonians) take the blocked two-sided Jacobi, shorter ones the
scalar Jacobi.  Every propagator equals the oracle's eigh-based one, on real, complex-embedded
and potential-only (degenerate) fibre Hamiltonians, and the blocked and scalar solvers agree."""
import numpy as np
import pytest

from oracle import splitting
from paper_2103_14897_amd import lsx
from paper_2103_14897_amd import workloads as wl

pytestmark = pytest.mark.gpu

ASYM1 = {(1,): 0.6 + 0.45j, (-1,): 0.6 - 0.45j, (2,): 0.2 - 0.1j, (-2,): 0.2 + 0.1j}
ASYM2 = {(1,): 0.5 - 0.3j, (-1,): 0.5 + 0.3j, (0,): 0.15}

CASES = [
    (wl.twisted_system(1500.0), 0.0, "exact"),          # real, lengths up to 199
    (wl.twisted_system(1500.0), 1.0, "exact"),          # potential-only windows, degenerate spectra
    (wl.chain_system(2.0e4, pot1=ASYM1, pot2=ASYM2), 0.0, "exact"),  # complex: embedded size 2L up to 206
    (wl.chain_system(2.0e4, pot1=ASYM1, pot2=ASYM2), 0.0, "cn"),
]
IDS = ["twisted-k0", "twisted-k1", "complex-chain", "complex-chain-cn"]


@pytest.mark.parametrize("spec,kappa,flow", CASES, ids=IDS)
def test_blocked_jacobi_propagators(monkeypatch, spec, kappa, flow):
    print(f"[case] eigensolver {spec.name} kappa={kappa} {flow}", flush=True)
    scheme = "strang_cn" if flow == "cn" else "strang"
    tau = 0.005
    S = lsx.System.from_spec(spec)
    O = splitting.Lifted.from_spec(spec)
    P = lsx.Plan(S, tau, scheme, kappa, "fp64")
    monkeypatch.setenv("LSX_BLOCKED_JACOBI", "0")
    P0 = lsx.Plan(S, tau, scheme, kappa, "fp64")
    monkeypatch.delenv("LSX_BLOCKED_JACOBI")
    try:
        plan = splitting.SplitPlan(O, kappa, flow)
        embed = 2 if any(complex(v).imag != 0 for v in list(spec.pot1.values()) + list(spec.pot2.values())) else 1
        nlong = 0
        for layer in (1, 2):
            ptr, _ = S.fibres(layer)
            L = np.diff(ptr)
            nlong += int((embed * L > 96).sum())
            for half, t in ((0, tau), (1, tau / 2)) if layer == 1 else ((0, tau),):
                ref = plan.propagators(layer, t)
                for f in range(S.nfibres[layer]):
                    # FP64 eigendecompositions (this library's and the oracle's) carry eigenvalue
                    # errors of about eps ||H||, i.e. phase errors of eps t ||H|| in exp(-i t lambda):
                    # the bar is 1e-13 up to t ||H|| = 10 and grows with it beyond
                    H = O.fibre_hamiltonian(layer, O.fib[layer][f][1], kappa)
                    tol = 1e-13 * max(1.0, t * np.abs(np.linalg.eigvalsh(H)).max() / 10.0)
                    got = P.propagator(layer, half, f)
                    assert np.abs(got - ref[f]).max() < tol, (layer, half, f, L[f], tol)
                    if embed * L[f] > 96:
                        assert np.abs(got - P0.propagator(layer, half, f)).max() < tol, (layer, f)
        assert nlong > 0
    finally:
        P.destroy()
        P0.destroy()
        S.destroy()
