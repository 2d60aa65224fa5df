"""Seeded synthetic inputs for the lifted layer-splitting step.

This module only *describes* workloads: lattice matrices, Fourier coefficients
of the two layer potentials, cutoffs, and seeded initial coefficient arrays.
It holds none of the method's arithmetic (no index-set enumeration, no
Hamiltonians, no propagators, no time stepping).  Both the CPU oracle's tests
and the HIP path's tests/bench draw their inputs from here, so that the two
sides see identical data without sharing any of the method's code.

Problem statement being described: two d-dimensional periodic layers with
lattices R_j = A_j Z^d, potentials v_j given by Fourier coefficients on the
reciprocal lattice 2 pi A_j^{-T} Z^d (Sec. 2, eqs. (2.1)-(2.2)), a plane-wave
energy cutoff Ec (Sec. 3), and initial plane-wave coefficients phi_mn(0)
(Sec. 3, eq. (3.2); Sec. 5 uses Gaussian-in-K data).

Workload recipes (all synthetic; the paper uses no dataset):

* ``tiny_chain``     -- 1D+1D, L1 = 1, L2 = golden mean, V_j = 2 v_j cos(2 pi x / L_j),
                        v1 = 1.0, v2 = 0.7, ball cutoff Ec = 200, one Gaussian
                        wavepacket sigma = 2, k0 = 0; tau = 0.01, T = 1, Strang.
* ``chain``          -- same lattices/potentials, Ec = 2e4, 64 wavepackets,
                        k0 ~ U[-10, 10] (seeded PCG64), sigma = 2; tau = 1e-3, T = 2.
* ``twisted``        -- two triangular lattices (constant 1) rotated by +-2.5 deg,
                        V_j = sum over the six first-shell reciprocal vectors of
                        v_j cos(G.x) (so each of the six coefficients is v_j),
                        v1 = 1.0, v2 = 0.5, ball cutoff Ec = 6500, 128 wavepackets,
                        sigma = 3, k0 area-uniform in |k0| <= 5; tau = 5e-3, T = 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN = (1.0 + math.sqrt(5.0)) / 2.0


@dataclass
class SystemSpec:
    """A two-layer incommensurate system (Sec. 2) plus its plane-wave cutoff (Sec. 3).

    ``A1``/``A2`` are d x d lattice matrices whose columns are the primitive
    vectors (R_j = A_j Z^d).  ``pot1``/``pot2`` map integer index tuples m to the
    complex Fourier coefficient v^(j)_m of eq. (2.2).  ``cutoff`` is ``"ball"``
    (|G1m|^2 + |G2n|^2 <= 2 Ec) or ``"product"`` (I1 x I2 of Sec. 3).
    """

    d: int
    A1: np.ndarray
    A2: np.ndarray
    Ec: float
    cutoff: str = "ball"
    pot1: dict = field(default_factory=dict)
    pot2: dict = field(default_factory=dict)
    name: str = ""

    def reciprocal(self, j: int) -> np.ndarray:
        """2 pi A_j^{-T} (columns are the reciprocal primitive vectors, Sec. 2)."""
        A = self.A1 if j == 1 else self.A2
        return 2.0 * math.pi * np.linalg.inv(A).T

    def pot_arrays(self, j: int):
        """(idx int32 [nv, d], re float64 [nv], im float64 [nv]) for layer j."""
        pot = self.pot1 if j == 1 else self.pot2
        keys = sorted(pot.keys())
        idx = np.array(keys, dtype=np.int32).reshape(len(keys), self.d)
        vals = np.array([complex(pot[k]) for k in keys], dtype=np.complex128)
        return idx, vals.real.copy(), vals.imag.copy()


def _cos_pot_1d(v: float) -> dict:
    # 2 v cos(2 pi x / L) = v e^{iGx} + v e^{-iGx}
    return {(1,): complex(v), (-1,): complex(v)}


def chain_system(Ec: float, L1: float = 1.0, L2: float = GOLDEN, v1: float = 1.0,
                 v2: float = 0.7, cutoff: str = "ball", pot1=None, pot2=None) -> SystemSpec:
    """1D+1D incommensurate chain (period ratio L2/L1)."""
    return SystemSpec(
        d=1,
        A1=np.array([[float(L1)]]),
        A2=np.array([[float(L2)]]),
        Ec=float(Ec),
        cutoff=cutoff,
        pot1=dict(pot1) if pot1 is not None else _cos_pot_1d(v1),
        pot2=dict(pot2) if pot2 is not None else _cos_pot_1d(v2),
        name=f"chain_Ec{Ec:g}",
    )


def _rot(theta: float) -> np.ndarray:
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s], [s, c]])


TRIANGULAR = np.array([[1.0, 0.5], [0.0, math.sqrt(3.0) / 2.0]])
# first shell of the triangular reciprocal lattice in index coordinates
FIRST_SHELL = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1)]


def twisted_system(Ec: float, theta_deg: float = 5.0, v1: float = 1.0, v2: float = 0.5,
                   cutoff: str = "ball", a: float = 1.0) -> SystemSpec:
    """Two triangular layers rotated by +theta/2 and -theta/2."""
    th = math.radians(theta_deg) / 2.0
    A1 = a * _rot(+th) @ TRIANGULAR
    A2 = a * _rot(-th) @ TRIANGULAR
    return SystemSpec(
        d=2, A1=A1, A2=A2, Ec=float(Ec), cutoff=cutoff,
        pot1={k: complex(v1) for k in FIRST_SHELL},
        pot2={k: complex(v2) for k in FIRST_SHELL},
        name=f"twisted{theta_deg:g}_Ec{Ec:g}",
    )


@dataclass
class MultiSpec:
    """A system of L >= 2 periodic layers (Sec. 2 with one lattice and potential per layer):
    ``As[j]`` is layer j's d x d lattice matrix (columns primitive vectors), ``pots[j]`` its
    Fourier coefficients, ``cutoff`` ball (sum_j |G_j m_j|^2 <= 2 Ec) or product."""

    d: int
    As: list
    Ec: float
    cutoff: str = "ball"
    pots: list = field(default_factory=list)
    name: str = ""

    @property
    def L(self) -> int:
        return len(self.As)


def chain_layers(Ec: float, periods=(1.0, GOLDEN, math.sqrt(2.0)), v=(1.0, 0.7, 0.5),
                 cutoff: str = "ball") -> MultiSpec:
    """1D chains of the given periods, layer j with potential 2 v_j cos(2 pi x / L_j) (the first
    len(periods) strengths are used)."""
    return MultiSpec(d=1, As=[np.array([[float(p)]]) for p in periods], Ec=float(Ec), cutoff=cutoff,
                     pots=[_cos_pot_1d(x) for _, x in zip(periods, v)], name=f"chain{len(periods)}_Ec{Ec:g}")


def twisted_layers(Ec: float, thetas_deg=(-2.5, 0.0, 2.5), v=(1.0, 0.5, 0.7), cutoff: str = "ball") -> MultiSpec:
    """Triangular layers rotated by the given angles (a twisted trilayer for three angles),
    first-shell potentials of strengths v_j."""
    return MultiSpec(d=2, As=[_rot(math.radians(t)) @ TRIANGULAR for t in thetas_deg], Ec=float(Ec), cutoff=cutoff,
                     pots=[{k: complex(x) for k in FIRST_SHELL} for _, x in zip(thetas_deg, v)],
                     name=f"twisted{len(thetas_deg)}_Ec{Ec:g}")


@dataclass
class BlockSpec:
    """A lifted system whose layers share index blocks: block b has embedding ``Rs[b]`` (D x dim_b,
    columns the wavevectors of its entries), ``groups`` lists the blocks of each cutoff group
    (sum over the group of |R_b m_b|^2 <= 2 Ec), ``layers[j]`` = (first block, end block) of the
    blocks layer j's potential couples, ``pots[j]`` its Fourier coefficients over those blocks."""

    Rs: list
    groups: list
    Ec: float
    layers: list
    pots: list
    name: str = ""


def example3_system(Ec: float, s1: float = 1.0, s2: float = 2.0,
                    beta: float = (math.sqrt(5.0) - 1.0) / 2.0) -> BlockSpec:
    """The quasi-one-dimensional system of Example 3 (Sec. 5):
    V = s1 cos^2(beta x) cos^2(pi y / 2) + s2 cos^2(x) cos^2(pi y / 2), incommensurate in x and
    periodic in y.  Blocks (m, p, n): m and n index the x-wavevectors 2 beta m and 2 n of the two
    factors, p the y-wavevector pi p; cutoff groups (m, n) and p; layer 1 couples (m, p), layer
    2 couples (p, n).  cos^2(a z) has coefficients 1/2 at 0 and 1/4 at +-2a."""
    a = {0: 0.5, 1: 0.25, -1: 0.25}
    p1 = {(k, q): s1 * a[k] * a[q] for k in a for q in a}
    p2 = {(q, k): s2 * a[k] * a[q] for k in a for q in a}
    Rs = [np.array([[2.0 * beta], [0.0]]), np.array([[0.0], [math.pi]]), np.array([[2.0], [0.0]])]
    return BlockSpec(Rs=Rs, groups=[[0, 2], [1]], Ec=float(Ec), layers=[(0, 2), (1, 3)], pots=[p1, p2],
                     name=f"example3_Ec{Ec:g}")


def draw_k0(W: int, d: int, seed: int = 0, kmax: float = 10.0) -> np.ndarray:
    """Seeded wavepacket centres k0 [W, d] (PCG64).

    1D: uniform in [-kmax, kmax]; 2D: area-uniform in the disk |k0| <= kmax.
    """
    rng = np.random.default_rng(seed)
    if d == 1:
        return rng.uniform(-kmax, kmax, size=(W, 1))
    u = rng.uniform(0.0, 1.0, size=W)
    ang = rng.uniform(0.0, 2.0 * math.pi, size=W)
    r = kmax * np.sqrt(u)
    return np.stack([r * np.cos(ang), r * np.sin(ang)], axis=1)


def gaussian_state(spec: SystemSpec, mn: np.ndarray, k0: np.ndarray, sigma: float) -> np.ndarray:
    """Initial coefficients c[i, w] ~ exp(-sigma^2 |K_i - k0_w|^2 / 2), each column unit-norm.

    ``mn`` is the [N, 2d] integer list of lifted indices (m, n); K_i = G1m + G2n
    is the lifted wavevector of the basis function e^{i(G1m+G2n).x} (Sec. 3).
    The unit-norm columns follow the generalised form of the Sec. 5 initial data.
    """
    d = spec.d
    B1, B2 = spec.reciprocal(1), spec.reciprocal(2)
    K = mn[:, :d].astype(np.float64) @ B1.T + mn[:, d:].astype(np.float64) @ B2.T
    k0 = np.asarray(k0, dtype=np.float64).reshape(-1, d)
    diff2 = ((K[:, None, :] - k0[None, :, :]) ** 2).sum(axis=2)
    c = np.exp(-0.5 * sigma * sigma * diff2).astype(np.complex128)
    c /= np.linalg.norm(c, axis=0, keepdims=True)
    return c


def decaying_state(spec: SystemSpec, mn: np.ndarray, k0: np.ndarray, sigma: float,
                   alpha: float) -> np.ndarray:
    """Gaussian in K times exp(-alpha(|G1m|^2+|G2n|^2)): data that decays in the lifted index,
    so truncation effects at the cutoff boundary are negligible."""
    d = spec.d
    B1, B2 = spec.reciprocal(1), spec.reciprocal(2)
    g1 = mn[:, :d].astype(np.float64) @ B1.T
    g2 = mn[:, d:].astype(np.float64) @ B2.T
    K = g1 + g2
    k0 = np.asarray(k0, dtype=np.float64).reshape(-1, d)
    diff2 = ((K[:, None, :] - k0[None, :, :]) ** 2).sum(axis=2)
    lift = (g1 ** 2).sum(axis=1) + (g2 ** 2).sum(axis=1)
    c = np.exp(-0.5 * sigma * sigma * diff2 - alpha * lift[:, None]).astype(np.complex128)
    c /= np.linalg.norm(c, axis=0, keepdims=True)
    return c


def random_state(N: int, W: int, seed: int = 0) -> np.ndarray:
    """Complex Gaussian coefficients [N, W], each column unit-norm (seeded PCG64)."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((N, W)) + 1j * rng.standard_normal((N, W))
    c /= np.linalg.norm(c, axis=0, keepdims=True)
    return c.astype(np.complex128)


def batch_specs(n1d: int = 240, n2d: int = 16, seed: int = 0):
    """The batched uneven systems (seeded PCG64), as (spec, tau) pairs: n1d 1D+1D chains with
    period ratio drawn from {golden mean, sqrt 2, sqrt 3} and Ec log-uniform in [1e3, 2e4]
    (tau = 1e-3), then n2d twisted triangular bilayers with twist uniform in [1, 6] deg and N
    log-uniform in [1e5, 4e5] (Ec = 6500 sqrt(N / 398821); tau = 5e-3)."""
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(n1d):
        ratio = [GOLDEN, math.sqrt(2.0), math.sqrt(3.0)][rng.integers(3)]
        Ec = float(np.exp(rng.uniform(np.log(1e3), np.log(2e4))))
        specs.append((chain_system(Ec, L2=ratio), 1e-3))
    for _ in range(n2d):
        theta = float(rng.uniform(1.0, 6.0))
        Ntarget = float(np.exp(rng.uniform(np.log(1e5), np.log(4e5))))
        specs.append((twisted_system(6500.0 * math.sqrt(Ntarget / 398821.0), theta_deg=theta), 5e-3))
    return specs


@dataclass
class Workload:
    """A system, a wavepacket batch recipe and a time grid."""

    spec: SystemSpec
    W: int
    sigma: float
    kmax: float
    tau: float
    T: float
    seed: int = 0
    scheme: str = "strang"

    @property
    def nsteps(self) -> int:
        return int(round(self.T / self.tau))

    def k0(self) -> np.ndarray:
        if self.W == 1 and self.kmax == 0.0:
            return np.zeros((1, self.spec.d))
        return draw_k0(self.W, self.spec.d, self.seed, self.kmax)

    def initial_state(self, mn: np.ndarray) -> np.ndarray:
        return gaussian_state(self.spec, mn, self.k0(), self.sigma)


def tiny_chain() -> Workload:
    """1D+1D, Ec = 200, one wavepacket, tau = 0.01 to T = 1 (Strang)."""
    return Workload(chain_system(200.0), W=1, sigma=2.0, kmax=0.0, tau=0.01, T=1.0)


def chain(Ec: float = 2.0e4, W: int = 64) -> Workload:
    """1D+1D, Ec = 2e4, 64 wavepackets, tau = 1e-3 to T = 2 (Strang)."""
    return Workload(chain_system(Ec), W=W, sigma=2.0, kmax=10.0, tau=1.0e-3, T=2.0)


def twisted(Ec: float = 6500.0, W: int = 128) -> Workload:
    """Twisted triangular bilayer (+-2.5 deg), Ec = 6500, 128 wavepackets, tau = 5e-3 to T = 1."""
    return Workload(twisted_system(Ec), W=W, sigma=3.0, kmax=5.0, tau=5.0e-3, T=1.0)


def uniforms(shape, seed: int = 0) -> np.ndarray:
    """Uniform [0, 1) draws (PCG64) for the sampling steps; passed to every implementation as data."""
    return np.random.default_rng(seed).random(shape)


def mlp_init(nin: int, width: int = 64, seed: int = 0) -> np.ndarray:
    """Initial parameters of the proposal network as one float32 vector, in the order
    W1 [nin, width], b1, W2 [width, width], b2, w3 [width], b3: weights normal with variance
    1 / fan_in (the output layer scaled by 0.1), biases zero."""
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal(nin * width) / math.sqrt(nin), np.zeros(width),
             rng.standard_normal(width * width) / math.sqrt(width), np.zeros(width),
             0.1 * rng.standard_normal(width) / math.sqrt(width), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)
