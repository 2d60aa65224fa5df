"""ctypes binding of liblsx.so (argument marshalling only).

Every function of ``include/lsx.h`` is exposed under the same name with the same
arguments; the classes ``System``, ``Plan`` and ``State`` only hold handles and
call those functions.  All computation happens in the HIP library; importing
this module does not load it, the first call does, and it raises if the library
has not been built (``python -m paper_2103_14897_amd.build``).

Device memory and streams may come from PyTorch: pass ``tensor.data_ptr()`` of a
contiguous complex128 CUDA tensor of shape [N, W] to ``State(..., dev_ptr=...)``
and ``torch.cuda.current_stream().cuda_stream`` as a stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

# the in-tree library; LSX_LIB names another build of it (the host-sanitized one for CPU tests)
LIB_PATH = os.environ.get("LSX_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblsx.so")

LSX_OK, LSX_E_INVALID, LSX_E_NOT_HERMITIAN, LSX_E_OOM, LSX_E_HIP, LSX_E_EIG, LSX_E_NONFINITE, LSX_E_STATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
CUTOFF = {"ball": 0, "product": 1}
SCHEME = {"lie": 0, "strang": 1, "lie_be": 2, "strang_cn": 3, "yoshida4": 4}
PRECISION = {"fp64": 0, "mix_fp32": 1, "mix_bf16x3": 2}
OBS_MASS, OBS_ENERGY, OBS_FIBRE_MASS_1, OBS_FIBRE_MASS_2, OBS_FIBRE_MASS_3 = 1, 2, 4, 8, 16

_lib = None

_p = C.c_void_p
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_dp = C.POINTER(C.c_double)

_SIGS = {
    "lsx_last_error": (C.c_char_p, []),
    "lsx_system_create": (C.c_int, [C.c_int32, _dp, _dp, C.c_double, C.c_int32,
                                    C.c_int32, _i32p, _dp, _dp, C.c_int32, _i32p, _dp, _dp, C.POINTER(_p)]),
    "lsx_system_create_layers": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(_dp), C.c_double, C.c_int32,
                                           _i32p, C.POINTER(_i32p), C.POINTER(_dp), C.POINTER(_dp),
                                           C.POINTER(_p)]),
    "lsx_system_create_blocks": (C.c_int, [C.c_int32, C.c_int32, _i32p, C.POINTER(_dp), _i32p, C.c_double,
                                           C.c_int32, _i32p, _i32p, _i32p, C.POINTER(_i32p), C.POINTER(_dp),
                                           C.POINTER(_dp), C.POINTER(_p)]),
    "lsx_system_layers": (C.c_int, [_p, C.POINTER(C.c_int32), _i64p]),
    "lsx_system_size": (C.c_int, [_p, _i64p, _i64p, _i64p]),
    "lsx_index_get": (C.c_int, [_p, _i32p]),
    "lsx_fibre_get": (C.c_int, [_p, C.c_int32, _i32p, _i32p]),
    "lsx_system_destroy": (C.c_int, [_p]),
    "lsx_plan_create": (C.c_int, [_p, C.c_double, C.c_int32, C.c_double, C.c_int32, _p, C.POINTER(_p)]),
    "lsx_plan_propagator": (C.c_int, [_p, C.c_int32, C.c_int32, C.c_int32, _dp, _p]),
    "lsx_plan_destroy": (C.c_int, [_p]),
    "lsx_state_create": (C.c_int, [_p, C.c_int32, _p, C.POINTER(_p)]),
    "lsx_state_upload": (C.c_int, [_p, _dp, _p]),
    "lsx_state_download": (C.c_int, [_p, _dp, _p]),
    "lsx_state_device_ptr": (C.c_int, [_p, C.POINTER(_p)]),
    "lsx_state_tuning": (C.c_int, [_p, C.c_int32, _i32p, _i32p, _dp]),
    "lsx_state_store_mode": (C.c_int, [_p, _i32p, _dp]),
    "lsx_state_prefetch": (C.c_int, [_p, C.c_int32, _i32p]),
    "lsx_state_destroy": (C.c_int, [_p]),
    "lsx_step": (C.c_int, [_p, _p, C.c_int64, _p]),
    "lsx_fibre_pass": (C.c_int, [_p, _p, C.c_int32, C.c_int32, C.c_int32, _p]),
    "lsx_phase": (C.c_int, [_p, _p, C.c_int32, _p]),
    "lsx_observables": (C.c_int, [_p, _p, C.c_uint32, _dp, _p]),
    "lsx_batch_create": (C.c_int, [C.POINTER(_p), C.POINTER(_p), C.c_int32, C.POINTER(_p)]),
    "lsx_batch_step": (C.c_int, [_p, C.c_int64, _p]),
    "lsx_batch_tuning": (C.c_int, [_p, C.c_int32, _i32p, _i32p, _dp, _i32p]),
    "lsx_batch_destroy": (C.c_int, [_p]),
    "lsx_si_step": (C.c_int, [_p, _p, C.c_int64, _p]),
    "lsx_sampler_create": (C.c_int, [_p, _p, C.c_int32, C.c_int32, C.c_double, C.POINTER(_p)]),
    "lsx_sampler_set_mlp": (C.c_int, [_p, _p]),
    "lsx_sampler_destroy": (C.c_int, [_p]),
    "lsx_rb_step": (C.c_int, [_p, _p, C.c_int64, _p]),
    "lsx_ss_step": (C.c_int, [_p, _p, C.c_int64, _p]),
    "lsx_sampler_weights": (C.c_int, [_p, C.c_int32, C.c_int32, _p, _p, _p, _p]),
    "lsx_sampler_features": (C.c_int, [_p, C.c_int32, _p, _p]),
    "lsx_sampler_increments": (C.c_int, [_p, C.c_int32, C.c_int32, _p, _p]),
    "lsx_mlp_create": (C.c_int, [C.c_int32, C.POINTER(_p)]),
    "lsx_mlp_nparams": (C.c_int, [_p, _i64p]),
    "lsx_mlp_set": (C.c_int, [_p, C.POINTER(C.c_float), _p]),
    "lsx_mlp_get": (C.c_int, [_p, C.POINTER(C.c_float), _p]),
    "lsx_mlp_forward": (C.c_int, [_p, _p, C.c_int64, _p, _p]),
    "lsx_mlp_backward": (C.c_int, [_p, _p, C.c_int64, _p, _p, _p]),
    "lsx_mlp_loss": (C.c_int, [_p, _p, _p, _p, C.c_int64, C.c_double, _p, _p, _p]),
    "lsx_mlp_adam": (C.c_int, [_p, _p, C.c_double, C.c_double, C.c_double, C.c_double, _p]),
    "lsx_mlp_train_step": (C.c_int, [_p, _p, C.c_int64, _p, _p, C.c_int64, C.c_double, C.c_double, C.c_double,
                                     C.c_double, C.c_double, _p, _p]),
    "lsx_mlp_destroy": (C.c_int, [_p]),
    "lsx_live_buffers": (C.c_int, [_i64p, _i64p]),
    "lsx_plan_sharing": (C.c_int, [_p, C.c_int32, _i32p, _i32p]),
    "lsx_plan_band": (C.c_int, [_p, C.c_int32, _dp, _i64p, _i64p, _i64p, _i64p]),
    "lsx_plan_fibre_band": (C.c_int, [_p, C.c_int32, C.c_int32, _i32p]),
    "lsx_system_symmetries": (C.c_int, [_p, _i32p, _i32p]),
    "lsx_observables_noalloc": (C.c_int, [_p, _p, C.c_int32, C.c_uint32, _p, _p]),
    "lsx_state_set_tuning": (C.c_int, [_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "lsx_state_set_store_mode": (C.c_int, [_p, C.c_int32]),
    "lsx_system_create_desc": (C.c_int, [_p, C.POINTER(_p)]),
    "lsx_index_size": (C.c_int, [_p, _i64p]),
    "lsx_fibre_info": (C.c_int, [_p, C.c_int32, _i64p, _i32p]),
    "lsx_plan_create_desc": (C.c_int, [_p, _p, _p, C.POINTER(_p)]),
    "lsx_state_wrap": (C.c_int, [_p, C.c_int32, _p, C.POINTER(_p)]),
}


class SystemDesc(C.Structure):
    """lsx_system_desc of include/lsx.h."""
    _fields_ = [("d", C.c_int32), ("A1", C.c_double * 4), ("A2", C.c_double * 4), ("Ec", C.c_double),
                ("cutoff", C.c_int32), ("nv", C.c_int32 * 2), ("v_idx", _i32p * 2), ("v_re", _dp * 2),
                ("v_im", _dp * 2)]


class PlanDesc(C.Structure):
    """lsx_plan_desc of include/lsx.h."""
    _fields_ = [("tau", C.c_double), ("scheme", C.c_int32), ("kappa", C.c_double), ("precision", C.c_int32),
                ("max_wavepackets", C.c_int32), ("band_tol", C.c_double)]


def live_buffers():
    """(count, bytes) of the device buffers the library holds (lsx_live_buffers)."""
    n, b = C.c_int64(), C.c_int64()
    _check(lib().lsx_live_buffers(C.byref(n), C.byref(b)))
    return n.value, b.value


class LsxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lsx error {code}: {msg}")
        self.code = code


def lib():
    """Load liblsx.so (once) and declare the C signatures."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: when PyTorch is installed its bundled
        # libamdhip64.so.7 is loaded first, so liblsx.so (same SONAME) binds to it and
        # torch streams / device pointers are valid in the library.
        try:
            import torch  # noqa: F401
        except ImportError:  # pragma: no cover
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2103_14897_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code):
    if code != LSX_OK:
        raise LsxError(code, lib().lsx_last_error().decode())


def _stream(s):
    if s is None:
        return None
    if hasattr(s, "cuda_stream"):
        return _p(s.cuda_stream)
    return _p(int(s))


def _dptr(a):
    return a.ctypes.data_as(_dp)


def _dev(x):
    """Device pointer argument: a torch tensor (its data_ptr), an int address, or None."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return _p(x.data_ptr())
    return _p(int(x))


def _lattice(A, d):
    return np.asfortranarray(np.asarray(A, dtype=np.float64).reshape(d, d)).ravel(order="F")


def _potential(pot, d):
    keys = sorted((pot or {}).keys())
    idx = np.ascontiguousarray(np.array(keys, dtype=np.int32).reshape(len(keys), d))
    vals = np.array([complex(pot[k]) for k in keys], dtype=np.complex128)
    return len(keys), idx, np.ascontiguousarray(vals.real), np.ascontiguousarray(vals.imag)


class System:
    """lsx_system: lattices, potentials and the lifted cutoff set (host only)."""

    def __init__(self, d, A1, A2, Ec, cutoff="ball", pot1=None, pot2=None):
        self.d = int(d)
        A1, A2 = _lattice(A1, d), _lattice(A2, d)
        self._keep = []
        args = []
        for pot in (pot1, pot2):
            n, idx, re, im = _potential(pot, d)
            self._keep += [idx, re, im]
            args += [n, idx.ctypes.data_as(_i32p), _dptr(re), _dptr(im)]
        h = _p()
        _check(lib().lsx_system_create(self.d, _dptr(A1), _dptr(A2), float(Ec), CUTOFF[cutoff], *args,
                                       C.byref(h)))
        self._finish(h)

    @classmethod
    def layers(cls, d, As, Ec, cutoff="ball", pots=None):
        """A system of len(As) = 2 or 3 layers (lsx_system_create_layers); pots[j] maps index
        tuples of length d to the Fourier coefficients of layer j's potential."""
        self = cls.__new__(cls)
        self.d = d = int(d)
        nl = len(As)
        pots = list(pots) if pots is not None else [{}] * nl
        if len(pots) != nl:
            raise ValueError("one potential per layer")
        mats = [_lattice(A, d) for A in As]
        parts = [_potential(p, d) for p in pots]
        self._keep = mats + [x for part in parts for x in part[1:]]
        h = _p()
        _check(lib().lsx_system_create_layers(
            d, nl, (_dp * nl)(*[_dptr(A) for A in mats]), float(Ec), CUTOFF[cutoff],
            (C.c_int32 * nl)(*[p[0] for p in parts]), (_i32p * nl)(*[p[1].ctypes.data_as(_i32p) for p in parts]),
            (_dp * nl)(*[_dptr(p[2]) for p in parts]), (_dp * nl)(*[_dptr(p[3]) for p in parts]), C.byref(h)))
        self._finish(h)
        return self

    @classmethod
    def blocks(cls, Rs, groups, Ec, layers, pots):
        """A system whose layers may share index blocks (lsx_system_create_blocks).  Rs[b] is
        block b's D x dim_b embedding, groups a list of block lists (one per cutoff group),
        layers a list of (first block, end block) ranges, pots[j] maps index tuples over layer
        j's blocks to Fourier coefficients."""
        self = cls.__new__(cls)
        Rs = [np.asarray(R, dtype=np.float64) for R in Rs]
        D = Rs[0].shape[0]
        nb = len(Rs)
        dims = (C.c_int32 * nb)(*[R.shape[1] for R in Rs])
        mats = [np.asfortranarray(R).ravel(order="F") for R in Rs]
        grp = [0] * nb
        for g, bl in enumerate(groups):
            for b in bl:
                grp[b] = g
        nl = len(layers)
        off = np.concatenate([[0], np.cumsum([R.shape[1] for R in Rs])])
        parts = [_potential(p, int(off[e] - off[s0])) for p, (s0, e) in zip(pots, layers)]
        self._keep = mats + [x for part in parts for x in part[1:]]
        self.d = D
        h = _p()
        _check(lib().lsx_system_create_blocks(
            D, nb, dims, (_dp * nb)(*[_dptr(A) for A in mats]), (C.c_int32 * nb)(*grp), float(Ec), nl,
            (C.c_int32 * nl)(*[int(s0) for s0, _ in layers]), (C.c_int32 * nl)(*[int(e - s0) for s0, e in layers]),
            (C.c_int32 * nl)(*[p[0] for p in parts]), (_i32p * nl)(*[p[1].ctypes.data_as(_i32p) for p in parts]),
            (_dp * nl)(*[_dptr(p[2]) for p in parts]), (_dp * nl)(*[_dptr(p[3]) for p in parts]), C.byref(h)))
        self._finish(h, int(off[-1]))
        return self

    def _finish(self, h, S=None):
        self.h = h
        nl = C.c_int32()
        nf = (C.c_int64 * 3)()
        _check(lib().lsx_system_layers(self.h, C.byref(nl), nf))
        N = C.c_int64()
        _check(lib().lsx_system_size(self.h, C.byref(N), None, None))
        self.N, self.nlayers = N.value, nl.value
        self.nfibres = {j + 1: nf[j] for j in range(self.nlayers)}
        self.S = S if S is not None else self.nlayers * self.d

    @classmethod
    def from_spec(cls, spec):
        return cls(spec.d, spec.A1, spec.A2, spec.Ec, spec.cutoff, spec.pot1, spec.pot2)

    @classmethod
    def from_desc(cls, d, A1, A2, Ec, cutoff="ball", pot1=None, pot2=None):
        """The same system through the descriptor form (lsx_system_create_desc)."""
        self = cls.__new__(cls)
        self.d = d = int(d)
        desc = SystemDesc()
        desc.d = d
        for k, A in enumerate((A1, A2)):
            a = _lattice(A, d)
            getattr(desc, "A%d" % (k + 1))[:len(a)] = list(a)
        desc.Ec = float(Ec)
        desc.cutoff = CUTOFF[cutoff]
        self._keep = []
        for j, pot in enumerate((pot1, pot2)):
            n, idx, re, im = _potential(pot, d)
            self._keep += [idx, re, im]
            desc.nv[j] = n
            desc.v_idx[j] = idx.ctypes.data_as(_i32p)
            desc.v_re[j] = _dptr(re)
            desc.v_im[j] = _dptr(im)
        h = _p()
        _check(lib().lsx_system_create_desc(C.byref(desc), C.byref(h)))
        self._finish(h)
        return self

    def symmetries(self):
        """Integer matrices M [nsym, nlayers, d, d] of the system's point symmetries."""
        n = C.c_int32()
        _check(lib().lsx_system_symmetries(self.h, C.byref(n), None))
        M = np.zeros((n.value, self.nlayers, self.d, self.d), dtype=np.int32)
        _check(lib().lsx_system_symmetries(self.h, C.byref(n), M.ctypes.data_as(_i32p)))
        return M

    def index_size(self):
        """|I| through lsx_index_size."""
        n = C.c_int64()
        _check(lib().lsx_index_size(self.h, C.byref(n)))
        return n.value

    def fibre_info(self, layer):
        """(number of fibres, int32 lengths) of `layer` through lsx_fibre_info."""
        nf = C.c_int64()
        _check(lib().lsx_fibre_info(self.h, int(layer), C.byref(nf), None))
        lengths = np.zeros(nf.value, dtype=np.int32)
        _check(lib().lsx_fibre_info(self.h, int(layer), C.byref(nf), lengths.ctypes.data_as(_i32p)))
        return nf.value, lengths

    def index(self):
        mn = np.zeros((self.N, self.S), dtype=np.int32)
        _check(lib().lsx_index_get(self.h, mn.ctypes.data_as(_i32p)))
        return mn

    def fibres(self, layer):
        ptr = np.zeros(self.nfibres[layer] + 1, dtype=np.int32)
        rows = np.zeros(self.N, dtype=np.int32)
        _check(lib().lsx_fibre_get(self.h, layer, ptr.ctypes.data_as(_i32p), rows.ctypes.data_as(_i32p)))
        return ptr, rows

    def destroy(self):
        if self.h:
            _check(lib().lsx_system_destroy(self.h))
            self.h = None


class Plan:
    """lsx_plan: one-time fibre eigendecomposition and propagators on the GPU."""

    def __init__(self, system, tau, scheme="strang", kappa=0.0, precision="fp64", stream=None,
                 max_wavepackets=None, band_tol=None):
        """band_tol: None or 0 the library's default, < 0 dense products, > 0 that tolerance."""
        self.system = system
        self.tau, self.scheme, self.kappa, self.precision = float(tau), scheme, float(kappa), precision
        h = _p()
        if max_wavepackets is None and band_tol is None:
            _check(lib().lsx_plan_create(system.h, self.tau, SCHEME[scheme], self.kappa, PRECISION[precision],
                                         _stream(stream), C.byref(h)))
        else:
            desc = PlanDesc(self.tau, SCHEME[scheme], self.kappa, PRECISION[precision], int(max_wavepackets or 0),
                            float(band_tol or 0.0))
            _check(lib().lsx_plan_create_desc(system.h, C.byref(desc), _stream(stream), C.byref(h)))
        self.h = h

    def band(self, layer, stored=False):
        """(tolerance in use, complex multiply-adds per column of one layer pass, the dense count),
        and with stored=True also (band entries of the stored propagators, their rows)."""
        tol, kept, dense, sk, sr = C.c_double(), C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().lsx_plan_band(self.h, int(layer), C.byref(tol), C.byref(kept), C.byref(dense), C.byref(sk),
                                   C.byref(sr)))
        if stored:
            return tol.value, kept.value, dense.value, sk.value, sr.value
        return tol.value, kept.value, dense.value

    def fibre_band(self, layer, fibre):
        """[nrb, 2] int32: first and one past the last multiplied fibre position per 16-row block."""
        ptr, _ = self.system.fibres(layer)
        L = int(ptr[fibre + 1] - ptr[fibre])
        out = np.zeros(((L + 15) // 16, 2), dtype=np.int32)
        _check(lib().lsx_plan_fibre_band(self.h, int(layer), int(fibre), out.ctypes.data_as(_i32p)))
        return out

    def sharing(self, layer):
        """(distinct propagators stored for `layer`, point symmetries shared over)."""
        nd, ns = C.c_int32(), C.c_int32()
        _check(lib().lsx_plan_sharing(self.h, int(layer), C.byref(nd), C.byref(ns)))
        return nd.value, ns.value

    def propagator(self, layer, half, fibre, stream=None):
        ptr, _ = self.system.fibres(layer)
        L = int(ptr[fibre + 1] - ptr[fibre])
        out = np.zeros((L, L), dtype=np.complex128)
        _check(lib().lsx_plan_propagator(self.h, layer, half, fibre, out.ctypes.data_as(_dp), _stream(stream)))
        return out

    def destroy(self):
        if self.h:
            _check(lib().lsx_plan_destroy(self.h))
            self.h = None


class State:
    """lsx_state: W wavepackets c[N][W] complex128 on the device."""

    def __init__(self, plan, W, dev_ptr=None):
        self.plan, self.W, self.N = plan, int(W), plan.system.N
        h = _p()
        if dev_ptr:
            _check(lib().lsx_state_wrap(plan.h, self.W, _p(dev_ptr), C.byref(h)))
        else:
            _check(lib().lsx_state_create(plan.h, self.W, None, C.byref(h)))
        self.h = h

    def set_tuning(self, layer, nb, ks, groups=0):
        """Pin `layer`'s tile shape and prefetch depth (lsx_state_set_tuning)."""
        _check(lib().lsx_state_set_tuning(self.h, int(layer), int(nb), int(ks), int(groups)))

    def set_store_mode(self, nontemporal):
        """Pin the pass output store mode (lsx_state_set_store_mode)."""
        _check(lib().lsx_state_set_store_mode(self.h, int(nontemporal)))

    def upload(self, c, stream=None):
        c = np.ascontiguousarray(np.asarray(c, dtype=np.complex128).reshape(self.N, self.W))
        _check(lib().lsx_state_upload(self.h, c.ctypes.data_as(_dp), _stream(stream)))
        self._pending = c  # the copy is stream-ordered: the source lives until the next upload

    def download(self, stream=None):
        out = np.zeros((self.N, self.W), dtype=np.complex128)
        _check(lib().lsx_state_download(self.h, out.ctypes.data_as(_dp), _stream(stream)))
        return out

    def device_ptr(self):
        p = _p()
        _check(lib().lsx_state_device_ptr(self.h, C.byref(p)))
        return p.value

    def step(self, nsteps, stream=None):
        _check(lib().lsx_step(self.plan.h, self.h, int(nsteps), _stream(stream)))

    def fibre_pass(self, layer, half=0, count=1, stream=None):
        _check(lib().lsx_fibre_pass(self.plan.h, self.h, int(layer), int(half), int(count), _stream(stream)))

    def phase(self, half=0, stream=None):
        _check(lib().lsx_phase(self.plan.h, self.h, int(half), _stream(stream)))

    def observables(self, mask=OBS_MASS | OBS_ENERGY, stream=None):
        sys = self.plan.system
        sizes = [(OBS_MASS, self.W), (OBS_ENERGY, self.W)]
        sizes += [(OBS_FIBRE_MASS_1 << j, sys.nfibres.get(j + 1, 0) * self.W) for j in range(3)]
        total = sum(n for bit, n in sizes if mask & bit)
        out = np.zeros(total, dtype=np.float64)
        code = lib().lsx_observables(self.plan.h, self.h, int(mask), _dptr(out), _stream(stream))
        _check(code)
        res, o = {}, 0
        names = {OBS_MASS: "mass", OBS_ENERGY: "energy", OBS_FIBRE_MASS_1: "fibre_mass_1",
                 OBS_FIBRE_MASS_2: "fibre_mass_2", OBS_FIBRE_MASS_3: "fibre_mass_3"}
        for bit, n in sizes:
            if mask & bit:
                v = out[o:o + n]
                res[names[bit]] = v.reshape(-1, self.W) if bit >= OBS_FIBRE_MASS_1 else v
                o += n
        return res

    def si_step(self, nsteps, stream=None):
        """Semi-implicit steps (Alg. 1) with the plan's tau."""
        _check(lib().lsx_si_step(self.plan.h, self.h, int(nsteps), _stream(stream)))

    def tuning(self, layer):
        """(nb, ks, pass_us) of the tile shape chosen for `layer`'s fibre passes."""
        nb, ks, us = C.c_int32(), C.c_int32(), C.c_double()
        _check(lib().lsx_state_tuning(self.h, int(layer), C.byref(nb), C.byref(ks), C.byref(us)))
        return nb.value, ks.value, us.value

    def prefetch(self, layer):
        """Groups of k-steps in flight per wave chosen for `layer` (0: library default)."""
        u = C.c_int32()
        _check(lib().lsx_state_prefetch(self.h, int(layer), C.byref(u)))
        return u.value

    def store_mode(self):
        """(nontemporal, (cycle_us ordinary, cycle_us non-temporal)) chosen for the pass outputs."""
        nt, us = C.c_int32(), (C.c_double * 2)()
        _check(lib().lsx_state_store_mode(self.h, C.byref(nt), us))
        return nt.value, (us[0], us[1])

    def destroy(self):
        if self.h:
            _check(lib().lsx_state_destroy(self.h))
            self.h = None


class Batch:
    """lsx_batch: several (plan, state) pairs stepped together by grouped launches."""

    def __init__(self, states):
        n = len(states)
        plans = (_p * n)(*[st.plan.h.value for st in states])
        sts = (_p * n)(*[st.h.value for st in states])
        h = _p()
        _check(lib().lsx_batch_create(plans, sts, n, C.byref(h)))
        self.h = h
        self.states = list(states)

    def step(self, nsteps, stream=None):
        _check(lib().lsx_batch_step(self.h, int(nsteps), _stream(stream)))

    def tuning(self, layer):
        """(nb, ks, pass_us, launch_mode) chosen for `layer`'s grouped passes (launch_mode: 0 one
        workgroup per tile, 1 persistent with tile queues, 2 persistent with a static stride)."""
        nb, ks, us, mode = C.c_int32(), C.c_int32(), C.c_double(), C.c_int32()
        _check(lib().lsx_batch_tuning(self.h, int(layer), C.byref(nb), C.byref(ks), C.byref(us), C.byref(mode)))
        return nb.value, ks.value, us.value, mode.value

    def destroy(self):
        if self.h:
            _check(lib().lsx_batch_destroy(self.h))
            self.h = None


class Mlp:
    """lsx_mlp: the width-64 tanh proposal network (FP32 parameters on the device).

    Array arguments are device pointers (torch tensors or int addresses)."""

    def __init__(self, nin):
        h = _p()
        _check(lib().lsx_mlp_create(int(nin), C.byref(h)))
        self.h, self.nin = h, int(nin)
        n = C.c_int64()
        _check(lib().lsx_mlp_nparams(self.h, C.byref(n)))
        self.nparams = n.value

    def set(self, theta, stream=None):
        t = np.ascontiguousarray(np.asarray(theta, dtype=np.float32).reshape(self.nparams))
        _check(lib().lsx_mlp_set(self.h, t.ctypes.data_as(C.POINTER(C.c_float)), _stream(stream)))
        self._pending = t  # stream-ordered copy: the source lives until the next set

    def get(self, stream=None):
        t = np.zeros(self.nparams, dtype=np.float32)
        _check(lib().lsx_mlp_get(self.h, t.ctypes.data_as(C.POINTER(C.c_float)), _stream(stream)))
        return t

    def forward(self, X, M, z, stream=None):
        _check(lib().lsx_mlp_forward(self.h, _dev(X), int(M), _dev(z), _stream(stream)))

    def backward(self, X, M, dz, grad, stream=None):
        _check(lib().lsx_mlp_backward(self.h, _dev(X), int(M), _dev(dz), _dev(grad), _stream(stream)))

    def loss(self, z, b, gptr, ngroups, eps, out, dz, stream=None):
        _check(lib().lsx_mlp_loss(self.h, _dev(z), _dev(b), _dev(gptr), int(ngroups), float(eps), _dev(out),
                                  _dev(dz), _stream(stream)))

    def adam(self, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(lib().lsx_mlp_adam(self.h, _dev(grad), float(lr), float(beta1), float(beta2), float(eps),
                                  _stream(stream)))

    def train_step(self, X, M, b, gptr, ngroups, eps, lr, out, beta1=0.9, beta2=0.999, adam_eps=1e-8,
                   stream=None):
        _check(lib().lsx_mlp_train_step(self.h, _dev(X), int(M), _dev(b), _dev(gptr), int(ngroups), float(eps),
                                        float(lr), float(beta1), float(beta2), float(adam_eps), _dev(out),
                                        _stream(stream)))

    def destroy(self):
        if self.h:
            _check(lib().lsx_mlp_destroy(self.h))
            self.h = None


class Sampler:
    """lsx_sampler: semi-implicit / random batch / stochastic splitting steps of one state.

    Array arguments are device pointers (torch tensors or int addresses)."""

    def __init__(self, state, p1, p2, eps=0.05):
        h = _p()
        _check(lib().lsx_sampler_create(state.plan.h, state.h, int(p1), int(p2), float(eps), C.byref(h)))
        self.h, self.state, self.p, self.eps = h, state, (int(p1), int(p2)), float(eps)
        self.mlp = None

    def set_mlp(self, mlp):
        _check(lib().lsx_sampler_set_mlp(self.h, mlp.h if mlp is not None else None))
        self.mlp = mlp

    def rb_step(self, u, nsteps, stream=None):
        _check(lib().lsx_rb_step(self.h, _dev(u), int(nsteps), _stream(stream)))

    def ss_step(self, u, nsteps, stream=None):
        _check(lib().lsx_ss_step(self.h, _dev(u), int(nsteps), _stream(stream)))

    def weights(self, layer, mode, z, u, wt, stream=None):
        _check(lib().lsx_sampler_weights(self.h, int(layer), int(mode), _dev(z), _dev(u), _dev(wt),
                                         _stream(stream)))

    def features(self, layer, X, stream=None):
        _check(lib().lsx_sampler_features(self.h, int(layer), _dev(X), _stream(stream)))

    def increments(self, layer, half, b, stream=None):
        _check(lib().lsx_sampler_increments(self.h, int(layer), int(half), _dev(b), _stream(stream)))

    def destroy(self):
        if self.h:
            _check(lib().lsx_sampler_destroy(self.h))
            self.h = None
