"""CPU tests of the C-ABI library: symbols, host-side index set and fibre tables, errors.

These run without a GPU: lsx_system_* is host-only code.  Index sets and fibre
tables are integer work and must equal the oracle's exactly.
"""
import ctypes
import json
import os
import re

import numpy as np
import pytest

from oracle import lifted
from paper_2103_14897_amd import lsx
from paper_2103_14897_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "lsx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lsx_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert len(names) >= 18
    L = ctypes.CDLL(lsx.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(lsx._SIGS), "binding and header disagree"


@pytest.mark.parametrize("spec", [wl.chain_system(200.0), wl.chain_system(2.0e4), wl.chain_system(971.0, cutoff="product"),
                                  wl.twisted_system(300.0), wl.twisted_system(300.0, cutoff="product"),
                                  wl.chain_system(500.0, L2=1.5)],
                         ids=["tiny", "chain", "product1d", "twisted", "product2d", "commensurate"])
def test_index_set_and_fibres_equal_oracle(spec):
    sys = lsx.System.from_spec(spec)
    mn = lifted.index_set(spec.A1, spec.A2, spec.Ec, spec.cutoff)
    assert sys.N == len(mn)
    assert np.array_equal(sys.index(), mn.astype(np.int32))
    for layer in (1, 2):
        fib = lifted.fibres(mn, layer)
        ptr, rows = sys.fibres(layer)
        assert sys.nfibres[layer] == len(fib)
        assert np.array_equal(ptr, np.cumsum([0] + [len(r) for _, r in fib]))
        assert np.array_equal(rows, np.concatenate([r for _, r in fib]))
    sys.destroy()


def test_twisted_full_size_index_set_and_fibres_equal_oracle():
    """Full-size twisted bilayer (Ec = 6500, N = 398821): the library's lifted index set and
    both fibre tables (Sec. 3, Fig. 3.1) equal the oracle's bit for bit, and the fibre-length
    statistics equal the stored ones (written by tests/golden/make_golden.py from the oracle)."""
    spec = wl.twisted_system(6500.0)
    sys = lsx.System.from_spec(spec)
    try:
        mn = lifted.index_set(spec.A1, spec.A2, spec.Ec, spec.cutoff)
        assert sys.N == len(mn) == 398821
        assert np.array_equal(sys.index(), mn.astype(np.int32))
        gold = json.load(open(os.path.join(ROOT, "tests", "golden", "index_sets.json")))["twisted"]
        for layer in (1, 2):
            fib = lifted.fibres(mn, layer)
            ptr, rows = sys.fibres(layer)
            assert sys.nfibres[layer] == len(fib) == gold[f"nfibres_{layer}"] == 889
            assert np.array_equal(ptr, np.cumsum([0] + [len(r) for _, r in fib]))
            assert np.array_equal(rows, np.concatenate([r for _, r in fib]))
            L = np.diff(ptr)
            assert int((L.astype(np.int64) ** 2).sum()) == gold[f"sum_L2_{layer}"]
            assert [int(L.min()), int(L.max())] == gold[f"minmax_L_{layer}"]
    finally:
        sys.destroy()


def test_errors():
    with pytest.raises(lsx.LsxError) as e:
        lsx.System(1, [[1.0]], [[0.0]], 100.0)
    assert e.value.code == lsx.LSX_E_INVALID
    with pytest.raises(lsx.LsxError) as e:
        lsx.System(1, [[1.0]], [[1.6]], -1.0)
    assert e.value.code == lsx.LSX_E_INVALID
    with pytest.raises(lsx.LsxError) as e:
        lsx.System(1, [[1.0]], [[1.6]], 100.0, pot1={(1,): 0.5 + 0.1j, (-1,): 0.5 + 0.1j})
    assert e.value.code == lsx.LSX_E_NOT_HERMITIAN
    with pytest.raises(lsx.LsxError) as e:
        lsx.System(1, [[1.0]], [[1.6]], 100.0, pot2={(2,): 0.3})
    assert e.value.code == lsx.LSX_E_NOT_HERMITIAN
    with pytest.raises(lsx.LsxError) as e:
        lsx.System(3, np.eye(3), np.eye(3), 100.0)
    assert e.value.code == lsx.LSX_E_INVALID
    # a Hermitian complex potential is accepted
    s = lsx.System(1, [[1.0]], [[1.6]], 100.0, pot1={(1,): 0.5 + 0.1j, (-1,): 0.5 - 0.1j})
    s.destroy()
    assert lsx.lib().lsx_system_destroy(None) == 0


@pytest.mark.parametrize("spec", [wl.chain_layers(150.0), wl.chain_layers(120.0, cutoff="product"),
                                  wl.twisted_layers(40.0), wl.twisted_layers(30.0, cutoff="product"),
                                  wl.chain_layers(300.0, periods=(1.0, wl.GOLDEN))],
                         ids=["chain3", "product3", "twisted3", "twisted3_product", "chain2_layers"])
def test_layered_index_set_and_fibres_equal_oracle(spec):
    """lsx_system_create_layers: lifted index set and every layer's fibre table equal the
    L-layer oracle's exactly."""
    from oracle import multilayer as ml
    sys = lsx.System.layers(spec.d, spec.As, spec.Ec, spec.cutoff, spec.pots)
    mn = ml.index_set(spec.As, spec.Ec, spec.cutoff)
    assert sys.nlayers == spec.L and sys.N == len(mn)
    assert np.array_equal(sys.index(), mn.astype(np.int32))
    for layer in range(1, spec.L + 1):
        fib = ml.fibres(mn, layer, spec.L, spec.d)
        ptr, rows = sys.fibres(layer)
        assert sys.nfibres[layer] == len(fib)
        assert np.array_equal(ptr, np.cumsum([0] + [len(r) for _, r in fib]))
        assert np.array_equal(rows, np.concatenate([r for _, r in fib]))
    # the last layer's fibres are contiguous runs of the canonical order
    assert np.array_equal(sys.fibres(spec.L)[1], np.arange(sys.N))
    sys.destroy()


def test_two_layers_through_create_layers_equal_create():
    spec = wl.twisted_system(300.0)
    a = lsx.System.from_spec(spec)
    b = lsx.System.layers(spec.d, [spec.A1, spec.A2], spec.Ec, spec.cutoff, [spec.pot1, spec.pot2])
    assert b.nlayers == 2 and a.nfibres == b.nfibres
    assert np.array_equal(a.index(), b.index())
    for layer in (1, 2):
        assert all(np.array_equal(x, y) for x, y in zip(a.fibres(layer), b.fibres(layer)))
    a.destroy()
    b.destroy()


def test_layered_errors():
    one = [[1.0]]
    for As in ([one], [one, one, one, one]):
        with pytest.raises(lsx.LsxError) as e:
            lsx.System.layers(1, As, 100.0)
        assert e.value.code == lsx.LSX_E_INVALID
    with pytest.raises(lsx.LsxError) as e:
        lsx.System.layers(1, [one, [[1.6]], [[1.3]]], 100.0, pots=[{}, {}, {(2,): 0.3}])
    assert e.value.code == lsx.LSX_E_NOT_HERMITIAN
    with pytest.raises(ValueError):
        lsx.System.layers(1, [one, [[1.6]], [[1.3]]], 100.0, pots=[{}, {}])
    # a cutoff whose candidate combinations exceed what could be indexed fails at once
    with pytest.raises(lsx.LsxError) as e:
        lsx.System.layers(2, [wl.TRIANGULAR] * 3, 3.0e5)
    assert e.value.code == lsx.LSX_E_INVALID


def _example3_args(Ec):
    spec = wl.example3_system(Ec)
    return spec.Rs, spec.groups, spec.Ec, spec.layers, spec.pots


@pytest.mark.parametrize("Ec", [40.0, 300.0])
def test_block_system_tables_equal_oracle(Ec):
    """lsx_system_create_blocks on Example 3 (blocks (m, p, n), cutoff groups (m, n) and p,
    layer 1 on (m, p), layer 2 on (p, n)): index set and fibre tables equal the block oracle."""
    from oracle import blocks
    Rs, groups, Ec, layers, pots = _example3_args(Ec)
    S = lsx.System.blocks(Rs, groups, Ec, layers, pots)
    O = blocks.example3(Ec)
    assert S.N == O.N and S.nlayers == 2 and S.S == 3
    assert np.array_equal(S.index(), O.mn.astype(np.int32))
    for layer in (1, 2):
        ptr, rows = S.fibres(layer)
        assert S.nfibres[layer] == len(O.fib[layer])
        assert np.array_equal(ptr, np.cumsum([0] + [len(r) for _, r in O.fib[layer]]))
        assert np.array_equal(rows, np.concatenate([r for _, r in O.fib[layer]]))
    S.destroy()


def test_block_system_reduces_to_the_layer_constructor():
    spec = wl.twisted_layers(30.0)
    a = lsx.System.layers(spec.d, spec.As, spec.Ec, spec.cutoff, spec.pots)
    from oracle import multilayer as ml
    b = lsx.System.blocks([ml.reciprocal(A) for A in spec.As], [[0, 1, 2]], spec.Ec, [(0, 1), (1, 2), (2, 3)],
                          spec.pots)
    assert a.nfibres == b.nfibres and np.array_equal(a.index(), b.index())
    for layer in (1, 2, 3):
        assert all(np.array_equal(x, y) for x, y in zip(a.fibres(layer), b.fibres(layer)))
    a.destroy()
    b.destroy()


def test_block_system_errors():
    Rs, groups, Ec, layers, pots = _example3_args(40.0)
    with pytest.raises(lsx.LsxError) as e:  # the last layer must couple the last block
        lsx.System.blocks(Rs, groups, Ec, [(1, 3), (0, 2)], pots[::-1])
    assert e.value.code == lsx.LSX_E_INVALID
    with pytest.raises(lsx.LsxError) as e:  # singular embedding
        lsx.System.blocks([np.zeros((2, 1))] + Rs[1:], groups, Ec, layers, pots)
    assert e.value.code == lsx.LSX_E_INVALID
    with pytest.raises(lsx.LsxError) as e:  # not Hermitian
        lsx.System.blocks(Rs, groups, Ec, layers, [pots[0], {(1, 0): 0.3}])
    assert e.value.code == lsx.LSX_E_NOT_HERMITIAN


@pytest.mark.parametrize("spec", [wl.chain_system(2.0e4), wl.twisted_system(300.0, cutoff="product")],
                         ids=["chain", "product2d"])
def test_descriptor_form_equals_flat_arguments(spec):
    """lsx_system_create_desc, lsx_index_size and lsx_fibre_info give the system, size and fibre
    lengths of the flat-argument calls (host-only work)."""
    a = lsx.System.from_spec(spec)
    b = lsx.System.from_desc(spec.d, spec.A1, spec.A2, spec.Ec, spec.cutoff, spec.pot1, spec.pot2)
    try:
        assert b.index_size() == a.N == b.N
        assert np.array_equal(a.index(), b.index())
        for layer in (1, 2):
            nf, lengths = b.fibre_info(layer)
            ptr, rows = a.fibres(layer)
            assert nf == a.nfibres[layer]
            assert np.array_equal(lengths, np.diff(ptr))
            assert np.array_equal(b.fibres(layer)[1], rows)
        with pytest.raises(lsx.LsxError) as e:
            b.fibre_info(3)
        assert e.value.code == lsx.LSX_E_INVALID
    finally:
        a.destroy()
        b.destroy()
    L = lsx.lib()
    assert L.lsx_system_create_desc(None, lsx.C.byref(lsx._p())) == lsx.LSX_E_INVALID
    assert L.lsx_index_size(None, None) == lsx.LSX_E_INVALID
    assert L.lsx_plan_create_desc(None, None, None, None) == lsx.LSX_E_INVALID
    assert L.lsx_state_wrap(None, 4, None, None) == lsx.LSX_E_INVALID
    assert L.lsx_state_set_tuning(None, 1, 1, 2, 0) == lsx.LSX_E_INVALID
    assert L.lsx_state_set_store_mode(None, 0) == lsx.LSX_E_INVALID


ASYM1 = {(1,): 0.6 + 0.45j, (-1,): 0.6 - 0.45j}


@pytest.mark.parametrize("spec,expect", [(wl.chain_system(2.0e4), 1), (wl.chain_system(500.0, L2=1.5), 1),
                                         (wl.twisted_system(300.0), 5), (wl.twisted_system(300.0, cutoff="product"), 5),
                                         (wl.twisted_system(600.0, theta_deg=3.0), 5),
                                         (wl.chain_system(971.0, pot1=ASYM1), 0)],
                         ids=["chain", "commensurate", "twisted", "product2d", "twist3", "complex-odd"])
def test_point_symmetries_map_the_oracle_system_onto_itself(spec, expect):
    """Every point symmetry the library reports (integer M_j per layer) maps the oracle's lifted
    index set onto itself, keeps every potential coefficient and |K|^2 (Secs. 2-3), and
    together with the identity the symmetries form a group.  Triangular lattices give the five
    non-trivial rotations by multiples of 60 degrees, 1D chains x -> -x, and a potential that
    is not even (complex coefficients) none."""
    S = lsx.System.from_spec(spec)
    try:
        M = S.symmetries()
    finally:
        S.destroy()
    assert M.shape[0] == expect
    d = spec.d
    mn = lifted.index_set(spec.A1, spec.A2, spec.Ec, spec.cutoff)
    K = lifted.lifted_wavevectors(spec.A1, spec.A2, mn)
    K2 = (K * K).sum(axis=1)
    keys = {tuple(r): i for i, r in enumerate(mn.tolist())}
    mats = [np.eye(d, dtype=np.int64)[None].repeat(2, 0)] + [M[e].astype(np.int64) for e in range(M.shape[0])]
    for Mg in mats[1:]:
        img = np.concatenate([mn[:, :d] @ Mg[0].T, mn[:, d:] @ Mg[1].T], axis=1)
        idx = np.array([keys.get(tuple(r), -1) for r in img.tolist()])
        assert np.all(idx >= 0) and len(set(idx.tolist())) == len(mn)
        assert np.allclose(K2[idx], K2, rtol=1e-12, atol=1e-9)
        for pot, Mj in ((spec.pot1, Mg[0]), (spec.pot2, Mg[1])):
            for m, v in pot.items():
                im = tuple(int(x) for x in Mj @ np.array(m))
                assert im in pot and abs(pot[im] - v) <= 1e-14 * max(abs(x) for x in pot.values())
    # closure: the product of two symmetries is the identity or another reported symmetry
    as_key = [tuple(Mg.ravel().tolist()) for Mg in mats]
    for A in mats:
        for B in mats:
            assert tuple(np.einsum("jab,jbc->jac", A, B).ravel().tolist()) in as_key


def test_point_symmetry_permutes_oracle_fibre_propagators():
    """The reading behind propagator sharing, checked on the oracle alone: for a symmetry
    (M_1, M_2), the layer-j fibre with fixed index M_k m_k has the fibre Hamiltonian of the
    fibre with fixed m_k with rows relabelled m_j -> M_j m_j (eq. 3.6), so its exact propagator
    is the same matrix permuted, for every kinetic share."""
    from oracle import splitting
    spec = wl.twisted_system(300.0)
    S = lsx.System.from_spec(spec)
    try:
        M = S.symmetries().astype(np.int64)
    finally:
        S.destroy()
    O = splitting.Lifted.from_spec(spec)
    d = spec.d
    keys = {tuple(r): i for i, r in enumerate(O.mn.tolist())}
    for kappa in (0.0, 0.5):
        plan = splitting.SplitPlan(O, kappa)
        for layer in (1, 2):
            props = plan.propagators(layer, 0.013)
            fib_of = {}
            for f, (_, rows) in enumerate(O.fib[layer]):
                for r in rows:
                    fib_of[int(r)] = f
            for f in (0, len(O.fib[layer]) // 3, len(O.fib[layer]) // 2):
                rows = O.fib[layer][f][1]
                for Mg in M:
                    img = np.concatenate([O.mn[rows, :d] @ Mg[0].T, O.mn[rows, d:] @ Mg[1].T], axis=1)
                    irows = np.array([keys[tuple(r)] for r in img.tolist()])
                    f2 = fib_of[int(irows[0])]
                    r2 = O.fib[layer][f2][1]
                    assert sorted(irows.tolist()) == r2.tolist()
                    pos = {int(r): a for a, r in enumerate(r2)}
                    perm = np.array([pos[int(r)] for r in irows])
                    P2 = props[f2][np.ix_(perm, perm)]
                    assert np.abs(P2 - props[f]).max() < 1e-13
