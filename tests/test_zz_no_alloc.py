"""The allocation-free observables entry point (lsx_observables_noalloc) through the C-ABI: its
device-resident results equal lsx_observables' bit for bit on two calls in a row, the second
with a smaller input, and a call whose reduction partials would not fit the static scratch is
refused before anything is launched."""
import ctypes as C

import numpy as np
import pytest

from paper_2103_14897_amd import lsx
from paper_2103_14897_amd import workloads as wl

pytestmark = pytest.mark.gpu

MASK = lsx.OBS_MASS | lsx.OBS_ENERGY | lsx.OBS_FIBRE_MASS_1 | lsx.OBS_FIBRE_MASS_2


def _noalloc(plan, c_dev, W, mask, nout):
    import torch

    out = torch.full((nout,), float("nan"), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    code = lsx.lib().lsx_observables_noalloc(plan.h, C.c_void_p(c_dev.data_ptr()), W, mask,
                                             C.c_void_p(out.data_ptr()), C.c_void_p(stream.cuda_stream))
    if code != lsx.LSX_OK:
        raise lsx.LsxError(code, lsx.lib().lsx_last_error().decode())
    stream.synchronize()
    return out.cpu().numpy()


def _reference(plan, c, W):
    st = lsx.State(plan, W)
    try:
        st.upload(c)
        r = st.observables(MASK)
    finally:
        st.destroy()
    return np.concatenate([r["mass"], r["energy"], r["fibre_mass_1"].ravel(), r["fibre_mass_2"].ravel()])


def test_noalloc_observables_equal_the_allocating_entry_point():
    import torch

    print("[case] no-alloc observables: chain Ec=2e4 W=64, then W=8, then chain Ec=971 W=5", flush=True)
    big = lsx.System.from_spec(wl.chain_system(2.0e4))
    small = lsx.System.from_spec(wl.chain_system(971.0))
    Pb = lsx.Plan(big, 1e-3, "strang", 0.0, "fp64")
    Ps = lsx.Plan(small, 1e-3, "strang", 0.0, "fp64")
    try:
        for plan, W, seed in ((Pb, 64, 1), (Pb, 8, 2), (Ps, 5, 3)):
            S = plan.system
            c = wl.random_state(S.N, W, seed=seed) * (1.0 + seed)
            ref = _reference(plan, c, W)
            c_dev = torch.from_numpy(c).to("cuda")
            torch.cuda.synchronize()
            nout = W * (2 + S.nfibres[1] + S.nfibres[2])
            got = _noalloc(plan, c_dev, W, MASK, nout)
            assert got.shape == ref.shape
            assert np.array_equal(got, ref), (S.N, W)
            # mass is the squared 2-norm of every column (eq. 2.3 via orthonormality)
            assert np.allclose(got[:W], (np.abs(c) ** 2).sum(axis=0), rtol=1e-13, atol=0)
            # a single block on its own lands at the start of the output
            only = _noalloc(plan, c_dev, W, lsx.OBS_FIBRE_MASS_2, W * S.nfibres[2])
            assert np.array_equal(only, ref[W * (2 + S.nfibres[1]):])
        # 21 partial blocks x 65536 wavepackets exceed the 2^20 doubles of scratch: refused on
        # the host (the tiny array passed is never read)
        dummy = torch.zeros(16, dtype=torch.complex128, device="cuda")
        out = torch.zeros(16, dtype=torch.float64, device="cuda")
        code = lsx.lib().lsx_observables_noalloc(Pb.h, C.c_void_p(dummy.data_ptr()), 65536, lsx.OBS_MASS,
                                                 C.c_void_p(out.data_ptr()), None)
        assert code == lsx.LSX_E_INVALID
        assert "static scratch" in lsx.lib().lsx_last_error().decode()
        assert torch.count_nonzero(out).item() == 0
    finally:
        for o in (Pb, Ps, big, small):
            o.destroy()
