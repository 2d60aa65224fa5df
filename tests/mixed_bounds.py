"""Rounding-error bounds of the mixed-precision fibre passes, derived from the arithmetic.

A mixed pass computes y = d .* x + E x~ for every fibre, with d = diag P and E = P - diag(d)
taken from the FP64 propagator P of the fibre, and the product formed on the matrix cores.
Against the exact FP64 pass y* = P x, with u = 2^-24 (FP32 unit roundoff) and
gamma_n = n u / (1 - n u) (standard model of floating-point summation):

FP32 path (E and x rounded to FP32, complex products in the three-real-product form
k1 = (a + b) c, k2 = a (d - c), k3 = b (c + d), FP32 accumulation over the fibre):
  * rounding E and x: |E~ - E| <= u |E|, |x~ - x| <= u |x|                        -> 2u
  * the sums a + b, d - c, c + d: one rounding each, on operands bounded by
    sqrt(2)|E| and sqrt(2)|x|                                                      -> 2u sqrt 2
  * accumulation of k1 and k3 (or k2) over L terms, plus the split-K reduction of the
    partial sums (at most 8 more additions): gamma_{L+8} on sums bounded by
    sqrt(2)|E| sqrt(2)|x| each, two sums per component                             -> 4 gamma_{L+8}
  * the final subtraction of two such sums in FP32                                 -> 2u sqrt 2
  per element |y - y*|_a <= c_L (|E| |x|)_a with c_L = 2u + 4 sqrt(2) u + 4 gamma_{L+8},
  times sqrt 2 for combining the real and imaginary parts.
BF16x3 path (E split into three bf16 terms by round-to-nearest-even with 8 significant bits,
remainder below 2^-24 |E|, |E1| <= 2^-9 |E|, |E2| <= 2^-18 |E|; x rounded to FP32 and then split
exactly into three bf16 terms by truncation, |x1| < 2^-7 |x|, |x2| < 2^-14 |x| (the row-split
kernel; the others split x by rounding, which is tighter); six of the nine cross products
kept, the dropped E1 x2, E2 x1, E2 x2 together below (2^-23 + 2^-25 + 2^-32) |E| |x| < 3u;
four real products per complex product, FP32 accumulation over 6 L terms):
  c_L = 2u + 3u + 2 gamma_{6L+8}, times sqrt 2.
In the 2-norm: ||y - y*|| <= sqrt(2) c_Lmax || |E| ||_2 ||x||, with |E| the entrywise modulus.

Band-limited products (lsx_plan_band): the passes leave out propagator chunks whose entries
all have |Re| + |Im| < tol (2^-44 by default on the mixed paths).  The left-out part B of a
fibre's E has at most L^2 entries below tol, so ||B||_2 <= ||B||_F <= L tol, which adds
Lmax tol to the relative bound of a pass.

Every pass is otherwise unitary (exact flows, FP64 diagonal and phase), so an error made in
one pass is carried by the later passes without growth: after a sequence of passes the
relative error against FP64 arithmetic is at most the sum of the per-pass bounds.  The FP64
path's own error (<= 1e-12 per step against the oracle) is added on top.
"""
import math

import numpy as np

U32 = 2.0 ** -24
BAND_TOL_MIXED = 2.0 ** -44  # the library's default band tolerance of the mixed paths


def gamma(n):
    return n * U32 / (1.0 - n * U32)


def pass_bound(props, precision, band_tol=BAND_TOL_MIXED):
    """Relative 2-norm error bound of one mixed pass with the fibre propagators ``props``,
    including the left-out band chunks (band_tol; 0 for dense products)."""
    worst = 0.0
    for P in props:
        L = P.shape[0]
        E = P - np.diag(np.diag(P))
        if L == 1 or not np.any(E):
            continue
        if precision == "mix_fp32":
            c = 2 * U32 + 4 * math.sqrt(2.0) * U32 + 4 * gamma(L + 8)
        elif precision == "mix_bf16x3":
            c = 5 * U32 + 2 * gamma(6 * L + 8)
        else:
            raise ValueError(precision)
        worst = max(worst, math.sqrt(2.0) * c * np.linalg.norm(np.abs(E), 2) + L * band_tol)
    return worst


def sequence_bound(plan, passes, precision):
    """Sum of the per-pass bounds over a list of (layer, t) fibre passes of an oracle plan."""
    cache = {}
    total = 0.0
    for layer, t in passes:
        key = (layer, float(t))
        if key not in cache:
            cache[key] = pass_bound(plan.propagators(layer, t), precision)
        total += cache[key]
    return total


def strang_passes(tau, nsteps, merged=True):
    """The passes of nsteps Strang steps: F1(tau/2) F2(tau) F1(tau/2) per step, with the two
    F1 halves between consecutive steps merged into one F1(tau) pass (merged=True, the
    library's exact-flow sequence) or applied separately (merged=False, Crank-Nicolson)."""
    if not merged:
        return [(1, tau / 2), (2, tau), (1, tau / 2)] * nsteps
    return [(1, tau / 2)] + [(2, tau), (1, tau)] * (nsteps - 1) + [(2, tau), (1, tau / 2)]


def lie_passes(tau, nsteps):
    return [(1, tau), (2, tau)] * nsteps
