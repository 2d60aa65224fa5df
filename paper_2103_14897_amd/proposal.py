"""Training data and training loop of the learned importance-sampling proposal.

Sequencing of liblsx calls only: the plain method advances the state (lsx_step), the sampler
writes per-fibre features and optimal-proposal targets b_f = ||(P_f - I) c_f||^2 of the
stochastic sub-steps (lsx_sampler_features / lsx_sampler_increments), and lsx_mlp_train_step
runs forward, objective, backward and Adam on the device.  Device buffers are torch tensors.
"""
from __future__ import annotations

import numpy as np

from . import lsx


def substep_layers(scheme: str):
    """(layer, propagator half) of the distinct stochastic sub-steps of a scheme: Strang samples
    F1(tau/2) and F2(tau), Lie F1(tau) and F2(tau)."""
    return [(1, 1), (2, 0)] if scheme in ("strang", "strang_cn") else [(1, 0), (2, 0)]


def collect(sampler, state, nsteps: int, every: int, stream=None):
    """Run the plain method `nsteps` steps on `state` and record, at step 0, every, 2 every, ...
    (before stepping on), the features X and targets b of every stochastic sub-step.

    Returns (X [M, nin] float32, b [M] float64, gptr [G + 1] int64) on the state's device, with
    one group per (snapshot, sub-step, wavepacket): the nf rows of that wavepacket's fibres."""
    import torch

    plan, sysm = state.plan, state.plan.system
    nin = sysm.d + 3
    W = state.W
    Xs, bs, sizes = [], [], []
    done = 0
    while True:
        for layer, half in substep_layers(plan.scheme):
            nf = sysm.nfibres[layer]
            X = torch.empty((W, nf, nin), dtype=torch.float32, device="cuda")
            b = torch.empty((W, nf), dtype=torch.float64, device="cuda")
            sampler.features(layer, X, stream)
            sampler.increments(layer, half, b, stream)
            Xs.append(X.reshape(-1, nin))
            bs.append(b.reshape(-1))
            sizes += [nf] * W
        if done + every > nsteps:
            break
        state.step(every, stream)
        done += every
    gptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return torch.cat(Xs), torch.cat(bs), torch.as_tensor(gptr, device="cuda")


def train(net, X, b, gptr, iters: int, lr: float = 3e-3, eps: float = 0.05, log_every: int = 50, stream=None):
    """Full-batch Adam on the normalised variance objective; returns [(iteration, objective)]
    read back every `log_every` iterations (the objective is evaluated before each update)."""
    import torch

    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    G = int(gptr.numel()) - 1
    M = int(X.shape[0])
    log = []
    for it in range(iters):
        net.train_step(X, M, b, gptr, G, eps, lr, out, stream=stream)
        if it % log_every == 0 or it == iters - 1:
            log.append((it, float(out[0].item())))
    return log


def objective(net, X, b, nf: int, eps: float, stream=None):
    """Normalised variance objective of the proposal (net, or uniform when None) on rows X with
    targets b grouped by consecutive runs of nf rows."""
    import torch

    M = int(X.shape[0])
    z = torch.zeros(M, dtype=torch.float32, device="cuda")
    if net is not None:
        net.forward(X, M, z, stream)
    gp = torch.arange(0, M + 1, nf, dtype=torch.int64, device="cuda")
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    dz = torch.zeros(M, dtype=torch.float32, device="cuda")
    scratch = net if net is not None else lsx.Mlp(X.shape[1])
    try:
        scratch.loss(z, b, gp, M // nf, eps, out, dz, stream)
        return float(out[0].item())
    finally:
        if net is None:
            scratch.destroy()
