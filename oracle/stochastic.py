"""Semi-implicit and random batch steps, and stochastic layer splitting with a learned
importance-sampling proposal (oracle; test infrastructure only).

Semi-implicit step (Alg. 1, Sec. 4.1): the kinetic part implicitly, both potentials explicitly,
    c' = (I + i tau D)^{-1} (c - i tau V^1 c - i tau V^2 c),
with V^j applied fibre by fibre (the block structure of Sec. 3).

Random batch step (Alg. 4): the same step with each potential applied only on a random subset of
p fibres of its layer, scaled by (number of fibres of the layer) / p, so that its expectation over
the subsets is the semi-implicit step.  The subset is drawn without replacement.  Reading: on a
ball index set the fibre counts replace |I_1| and |I_2|.  Every column of c is an independent
realisation with its own subsets.

Stochastic layer splitting (the same sampling idea applied to the exact fibre flows): a layer
sub-step F_j(t) c = c + sum_f (P_f(t) - I) c_f is estimated from p fibres drawn independently
(with replacement) from a proposal q over the fibres of layer j:
    S_j c = c + sum_{s=1..p} (P_{f_s}(t) - I) c_{f_s} / (p q_{f_s}),
which is unbiased for any q with q_f > 0.  Uniform q_f = 1/n_f gives the weight n_f / p of Alg. 4.
For p iid draws the mean squared deviation per column is
    E || S_j c - F_j c ||^2 = (1/p) (sum_f b_f / q_f - sum_f b_f),   b_f = ||(P_f - I) c_f||^2,
minimised by q_f proportional to sqrt(b_f) (Cauchy-Schwarz).  The proposal is
q = (1 - eps) softmax(z) + eps / n_f with logits z from a small MLP of per-fibre features (fibre
Bloch shift and current fibre mass); the eps share keeps every q_f > 0 (defensive mixture).
Training minimises the normalised variance objective
    l(q) = sum_f b_f / q_f / (sum_f sqrt(b_f))^2   (>= 1, = 1 at the optimum when eps = 0)
averaged over groups (one group = one column of one layer sub-step), with Adam (Kingma & Ba).
The paper gives the random batch idea without analysis; the proposal and its objective are this
project's extension of it.
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------- semi-implicit / random batch


def _as2(c):
    c = np.asarray(c, dtype=np.complex128)
    return c.reshape(c.shape[0], -1)


def potential_apply(sys, layer: int, c: np.ndarray, weights=None) -> np.ndarray:
    """(V^j c) fibre by fibre; with ``weights`` [n_f, W] the fibre block f of column w is scaled by
    weights[f, w] (zero skips the fibre)."""
    c = _as2(c)
    out = np.zeros_like(c)
    for f, (_, rows) in enumerate(sys.fib[layer]):
        if weights is not None and not np.any(weights[f]):
            continue
        V = sys.fibre_hamiltonian(layer, rows, 1.0)  # kinetic share 1: the potential block alone
        y = V @ c[rows]
        out[rows] = y if weights is None else y * weights[f][None, :]
    return out


def semi_implicit_step(sys, c: np.ndarray, tau: float, a1=None, a2=None) -> np.ndarray:
    """One step of Alg. 1 (a1 = a2 = None) or of Alg. 4 (per-fibre, per-column weights a_j)."""
    c = _as2(c)
    psi1 = 1j * tau * potential_apply(sys, 1, c, a1)
    psi2 = 1j * tau * potential_apply(sys, 2, c, a2)
    return (c - psi1 - psi2) / (1.0 + 1j * tau * 0.5 * sys.K2)[:, None]


def subset_weights(nf: int, p: int, u: np.ndarray) -> np.ndarray:
    """Random subsets of p of the nf fibres, one per column, as weights [nf, W] (nf/p on the chosen
    fibres).  Column w is drawn by a partial Fisher-Yates shuffle with the uniforms u[w, 0..p-1]:
    position s swaps with s + floor(u (nf - s)), so every ordered p-tuple of distinct fibres is
    equally likely."""
    u = np.asarray(u, dtype=np.float64)
    if not 1 <= p <= nf:
        raise ValueError("need 1 <= p <= number of fibres")
    wt = np.zeros((nf, u.shape[0]))
    for w in range(u.shape[0]):
        perm = list(range(nf))
        for s in range(p):
            j = min(s + int(np.floor(u[w, s] * (nf - s))), nf - 1)
            perm[s], perm[j] = perm[j], perm[s]
        wt[perm[:p], w] = nf / p
    return wt


def random_batch_step(sys, c, tau, p1: int, u1, p2: int, u2) -> np.ndarray:
    """Alg. 4: p1 of the layer-1 fibres (uniforms u1 [W, p1]) and p2 of the layer-2 fibres."""
    a1 = subset_weights(len(sys.fib[1]), p1, u1)
    a2 = subset_weights(len(sys.fib[2]), p2, u2)
    return semi_implicit_step(sys, c, tau, a1, a2)


# ---------------------------------------------------------------- proposal and sampling


def proposal(z, nf: int, W: int, eps: float) -> np.ndarray:
    """q [W, nf] = (1 - eps) softmax(z[w]) + eps / nf per column; z None means uniform."""
    if z is None:
        return np.full((W, nf), 1.0 / nf)
    z = np.asarray(z, dtype=np.float64).reshape(W, nf)
    e = np.exp(z - z.max(axis=1, keepdims=True))
    return (1.0 - eps) * e / e.sum(axis=1, keepdims=True) + eps / nf


def draw(q: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Inverse-CDF draws: for column w and uniform u, the first f with cumsum(q[w])[f] > u
    (the last fibre when rounding leaves the total below u)."""
    W, nf = q.shape
    out = np.empty(u.shape, dtype=np.int64)
    for w in range(W):
        cdf = np.cumsum(q[w])
        out[w] = np.minimum(np.searchsorted(cdf, u[w], side="right"), nf - 1)
    return out


def draw_weights(q: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Importance weights [nf, W]: each of the p draws of column w adds 1 / (p q_f) to its fibre."""
    W, nf = q.shape
    p = u.shape[1]
    f = draw(q, u)
    wt = np.zeros((nf, W))
    for w in range(W):
        for s in range(p):
            wt[f[w, s], w] += 1.0 / (p * q[w, f[w, s]])
    return wt


def sampled_pass(plan, layer: int, t: float, c: np.ndarray, wt: np.ndarray) -> np.ndarray:
    """c + sum_f wt[f, w] ((P_f(t) c_f) - c_f): the weighted fibre increments of one layer."""
    c = _as2(c)
    out = c.copy()
    for f, ((_, rows), P) in enumerate(zip(plan.sys.fib[layer], plan.propagators(layer, t))):
        if not np.any(wt[f]):
            continue
        x = c[rows]
        out[rows] = x + wt[f][None, :] * (P @ x - x)
    return out


def increments(plan, layer: int, t: float, c: np.ndarray) -> np.ndarray:
    """b [W, nf] = ||(P_f(t) - I) c_f||^2 per column and fibre."""
    c = _as2(c)
    b = np.zeros((c.shape[1], len(plan.sys.fib[layer])))
    for f, ((_, rows), P) in enumerate(zip(plan.sys.fib[layer], plan.propagators(layer, t))):
        dx = P @ c[rows] - c[rows]
        b[:, f] = (dx.real ** 2 + dx.imag ** 2).sum(axis=0)
    return b


def substeps(scheme: str, tau: float):
    """Fibre sub-steps of one step in time order as (layer, t, t_phase): the layer sub-step of
    duration t, then a kinetic phase of duration t_phase (none when 0).  Lie: F1(tau), phase(tau),
    F2(tau); Strang: F1(tau/2), phase(tau/2), F2(tau), phase(tau/2), F1(tau/2)."""
    if scheme == "lie":
        return [(1, tau, tau), (2, tau, 0.0)]
    return [(1, tau / 2, tau / 2), (2, tau, tau / 2), (1, tau / 2, 0.0)]


def stochastic_step(plan, c, tau: float, scheme: str, u: np.ndarray, logits_fn=None, eps: float = 0.05):
    """One stochastic Lie or Strang step (unmerged).  u [nsub, W, p]: uniforms of each sub-step.
    logits_fn(layer, c) -> z [W, nf] (None: uniform proposal).  The proposal of each sub-step is
    computed from the state entering that sub-step."""
    c = _as2(c)
    for k, (layer, t, tph) in enumerate(substeps(scheme, tau)):
        nf = len(plan.sys.fib[layer])
        z = None if logits_fn is None else logits_fn(layer, c)
        q = proposal(z, nf, c.shape[1], eps)
        c = sampled_pass(plan, layer, t, c, draw_weights(q, u[k]))
        if tph != 0.0 and plan.kappa != 0.0:
            c = plan.apply_phase(c, tph)
    return c


# ---------------------------------------------------------------- features and MLP

def fibre_shifts(sys, layer: int) -> np.ndarray:
    """Bloch shift of every fibre of ``layer``: G_2 n for the layer-1 fibre of n, G_1 m for the
    layer-2 fibre of m (Sec. 3), with G_j = 2 pi A_j^{-T}."""
    keys = np.array([k for k, _ in sys.fib[layer]], dtype=np.float64).reshape(-1, sys.d)
    A = sys.A2 if layer == 1 else sys.A1
    B = 2.0 * np.pi * np.linalg.inv(A).T
    return keys @ B.T


def n_features(d: int) -> int:
    return d + 3


def features(sys, layer: int, c: np.ndarray) -> np.ndarray:
    """X [W, nf, d+3] per column and fibre: shift / Kmax (d entries), |shift|^2 / Kmax^2,
    log10(max(fibre mass, 1e-30)) / 10, and the layer sign (-1 for layer 1, +1 for layer 2);
    Kmax = sqrt(2 Ec)."""
    c = _as2(c)
    W = c.shape[1]
    fib = sys.fib[layer]
    kmax = np.sqrt(2.0 * sys.Ec)
    s = fibre_shifts(sys, layer) / kmax
    mass = np.array([(np.abs(c[rows]) ** 2).sum(axis=0) for _, rows in fib])  # [nf, W]
    X = np.zeros((W, len(fib), sys.d + 3))
    X[:, :, :sys.d] = s[None, :, :]
    X[:, :, sys.d] = (s * s).sum(axis=1)[None, :]
    X[:, :, sys.d + 1] = np.log10(np.maximum(mass.T, 1e-30)) / 10.0
    X[:, :, sys.d + 2] = -1.0 if layer == 1 else 1.0
    return X


def mlp_unpack(theta: np.ndarray, nin: int, H: int):
    """Flat parameter vector -> (W1 [nin, H], b1 [H], W2 [H, H], b2 [H], w3 [H], b3 scalar)."""
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = theta[o:o + nin * H].reshape(nin, H); o += nin * H
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    b3 = theta[o]
    return W1, b1, W2, b2, w3, b3


def mlp_size(nin: int, H: int) -> int:
    return nin * H + H + H * H + H + H + 1


def mlp_forward(theta, X: np.ndarray, H: int = 64):
    """Logits z = w3 . tanh(W2^T tanh(W1^T x + b1) + b2) + b3 for every row x of X [M, nin]."""
    X = np.asarray(X, dtype=np.float64).reshape(-1, np.shape(X)[-1])
    W1, b1, W2, b2, w3, b3 = mlp_unpack(theta, X.shape[1], H)
    h1 = np.tanh(X @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    return h2 @ w3 + b3


def mlp_backward(theta, X: np.ndarray, dz: np.ndarray, H: int = 64) -> np.ndarray:
    """Gradient of sum_m dz_m z_m with respect to the flat parameters (chain rule, tanh' = 1 - tanh^2)."""
    X = np.asarray(X, dtype=np.float64).reshape(-1, np.shape(X)[-1])
    dz = np.asarray(dz, dtype=np.float64).reshape(-1)
    W1, b1, W2, b2, w3, b3 = mlp_unpack(theta, X.shape[1], H)
    h1 = np.tanh(X @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    dw3 = h2.T @ dz
    db3 = dz.sum()
    da2 = (dz[:, None] * w3[None, :]) * (1.0 - h2 * h2)
    dW2 = h1.T @ da2
    db2 = da2.sum(axis=0)
    da1 = (da2 @ W2.T) * (1.0 - h1 * h1)
    dW1 = X.T @ da1
    db1 = da1.sum(axis=0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dw3, [db3]])


def proposal_loss(z: np.ndarray, b: np.ndarray, gptr: np.ndarray, eps: float):
    """Normalised variance objective and its gradient with respect to the logits.

    Groups g are the rows gptr[g]..gptr[g+1] of z and b.  Per group with sum b > 0:
    l_g = sum_f b_f / q_f / (sum_f sqrt b_f)^2, q = (1 - eps) softmax(z_g) + eps / n_g.
    Returns (mean of l_g over those groups, dL/dz [M], per-group l_g (0 for skipped groups))."""
    z = np.asarray(z, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    G = len(gptr) - 1
    lg = np.zeros(G)
    dz = np.zeros_like(z)
    active = 0
    for g in range(G):
        sl = slice(gptr[g], gptr[g + 1])
        bg = b[sl]
        if not bg.sum() > 0.0:
            continue
        active += 1
        n = bg.size
        e = np.exp(z[sl] - z[sl].max())
        sig = e / e.sum()
        q = (1.0 - eps) * sig + eps / n
        S = np.sqrt(bg).sum() ** 2
        lg[g] = (bg / q).sum() / S
        r = bg / (q * q)
        dz[sl] = (1.0 - eps) / S * sig * ((r * sig).sum() - r)
    if active == 0:
        return 0.0, dz, lg
    return lg.sum() / active, dz / active, lg


def adam_step(theta, m, v, g, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Alg. 1) at step t >= 1; returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
