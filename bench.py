"""Benchmark of the lifted layer-splitting step on one MI355X.

Workload (the configuration the coeff*steps/s metric is quoted on): two 1D layers
L1 = 1, L2 = golden mean, V_j = 2 v_j cos(2 pi x / L_j) with v1 = 1.0, v2 = 0.7,
ball cutoff Ec = 2e4 (N = 5149 lifted coefficients, 103 + 63 fibres of length
9-103), 64 Gaussian wavepackets (sigma = 2, k0 ~ U[-10, 10], seed 0), Strang layer
splitting with tau = 1e-3 to T = 2 (2000 steps).  Synthetic inputs, resident in
HBM before the timed region.

A step is one full Strang step (two fibre passes: layer 2 with tau, layer 1 with
tau; the half steps of consecutive steps are merged).  coeff*steps/s =
N * W * steps / (time of the timed steps).  Every precision path (plain FP64,
FP32 MFMA on the off-diagonal propagator part, BF16x3 split products) is timed;
the headline `value` is the fastest path whose relative L2 error after T against
the FP64 path is <= 1e-6.  The CPU oracle is timed on a bounded sample of the
same workload on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2103_14897_amd import lsx  # noqa: E402
from paper_2103_14897_amd import workloads as wl  # noqa: E402

PEAK = {"fp64": 78.6e12, "mix_fp32": 157.3e12, "mix_bf16x3": 2.5e15}
HBM_PEAK = 8.0e12
# bytes of propagator storage per fibre-matrix entry, per precision path (FP64: P in
# complex128; mixed: off-diagonal E in complex64 or three bf16 terms x (re, im))
PROP_BYTES = {"fp64": 16, "mix_fp32": 8, "mix_bf16x3": 12}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fibre_pass_chain_Ec2e4_W64_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2103_14897_amd", "csrc", "lsx_kernels.hip")


def measured_traffic(path):
    """HBM bytes per launch of the layer-2 pass from the committed rocprofv3 counters,
    or None when the kernel source has changed since they were taken."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
        h = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    if rec.get("kernel_source_sha256_16") != h or path not in rec.get("layer2_pass", {}):
        return None
    return rec["layer2_pass"][path]["hbm_bytes_per_launch"]
DTYPE = {"fp64": "f64", "mix_fp32": "f32-mfma+f64", "mix_bf16x3": "bf16x3-mfma+f64"}
METRIC = "coeff·steps/s, plain FP64 vs mixed at ≤1e-6 L2 error; % HBM/MFMA peak"


def cpu_baseline(spec, c0, tau, budget_s=15.0):
    """The CPU oracle (FP64 NumPy) on a bounded sample of the same workload."""
    from oracle import splitting
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = 1
    O = splitting.Lifted.from_spec(spec)
    plan = splitting.SplitPlan(O, 0.0)
    t0 = time.perf_counter()
    for layer in (1, 2):
        plan.propagators(layer, tau)
    plan.propagators(1, tau / 2)
    pre = time.perf_counter() - t0
    c = c0.copy()
    t0 = time.perf_counter()
    c = plan.strang_step(c, tau)
    one = time.perf_counter() - t0
    n = int(max(3, min(2000, budget_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    for _ in range(n):
        c = plan.strang_step(c, tau)
    el = time.perf_counter() - t0
    out = {"value": O.N * c0.shape[1] * n / el, "unit": "coeff*steps/s", "cores": int(threads),
           "kind": "oracle",
           "sample": f"{n} unmerged Strang steps of the same workload (N={O.N}, W={c0.shape[1]}), "
                     f"precompute {pre:.2f}s excluded"}
    # the same sample on one host thread, a third of the budget
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            n1 = max(3, n // 3)
            t0 = time.perf_counter()
            for _ in range(n1):
                c = plan.strang_step(c, tau)
            out["single_thread_value"] = O.N * c0.shape[1] * n1 / (time.perf_counter() - t0)
            out["single_thread_steps"] = n1
    except Exception:  # pragma: no cover
        pass
    return out


def batch_workload(args):
    """Many uneven systems in one grouped launch per pass, against stepping them one by one.

    Systems (seeded PCG64): `--batch-1d` 1D+1D chains with period ratio drawn from
    {golden mean, sqrt 2, sqrt 3} and Ec log-uniform in [1e3, 2e4], plus `--batch-2d`
    twisted triangular bilayers with twist uniform in [1, 6] deg and N log-uniform in
    [1e5, 4e5] (Ec = 6500 sqrt(N / 398821)); 16 wavepackets each; kinetic share `--kappa`
    (0: the paper's split, every fibre its own Bloch-shifted Hamiltonian, propagators shared
    over the point symmetries; 1: potential-only windows shared by translation), Strang,
    tau = 1e-3 (1D) / 5e-3 (2D), `--paths` first entry as precision.

    Roofline of each layer's grouped pass (time from the batch tuner's measurement): bytes =
    every system's state read and written (2 N W 16) plus its distinct propagators (and the FP64
    diagonal, 16 N, on the mixed paths); flops = 8 W sum L^2 over every fibre.
    """
    import torch
    prec = args.paths.split(",")[0]
    specs = wl.batch_specs(args.batch_1d, args.batch_2d)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    items = []
    for spec, tau in specs:
        S = lsx.System.from_spec(spec)
        P = lsx.Plan(S, tau, "strang", args.kappa, prec, stream)
        st = lsx.State(P, 16)
        st.upload(wl.random_state(S.N, 16, seed=len(items)), stream)
        items.append((S, P, st))
    pre = time.perf_counter() - t0
    print(f"[bench] batch: {len(items)} systems built in {pre:.1f} s", file=sys.stderr, flush=True)
    # algorithmic work of one grouped pass per layer, over all systems
    work = {1: [0.0, 0.0], 2: [0.0, 0.0]}
    distinct = {1: 0, 2: 0}
    for S, P, st in items:
        for j in (1, 2):
            L = np.diff(S.fibres(j)[0]).astype(np.int64)
            nd = P.sharing(j)[0]
            distinct[j] += nd
            # band-limited products (lsx_plan_band): the entries inside the bands; bytes count the
            # stored propagators once (each orbit or window class stores one) and their diagonals
            _, kept, _, skept, srows = P.band(j, stored=True)
            work[j][0] += 8.0 * 16 * kept
            work[j][1] += 2.0 * S.N * 16 * 16 + PROP_BYTES[prec] * skept + (16.0 * srows if prec != "fp64" else 0.0)
    B = lsx.Batch([it[2] for it in items])
    coeffs = sum(it[0].N * 16 for it in items)
    B.step(args.warmup, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    B.step(args.steps, stream)
    e1.record(stream)
    e1.synchronize()
    ms_batch = e0.elapsed_time(e1)
    e0.record(stream)
    for it in items:
        it[2].step(args.steps, stream)
    e1.record(stream)
    e1.synchronize()
    ms_seq = e0.elapsed_time(e1)
    roof = {}
    for j in (1, 2):
        us = B.tuning(j)[2]
        if us > 0:
            gbs = work[j][1] / (us * 1e-6) / 1e9
            tfs = work[j][0] / (us * 1e-6) / 1e12
            roof[f"layer{j}"] = {"pass_us": us, "GB/s": gbs, "hbm_frac": gbs * 1e9 / HBM_PEAK, "TFLOP/s": tfs,
                                 "mfma_frac": tfs * 1e12 / PEAK[prec], "algorithmic_bytes": work[j][1],
                                 "algorithmic_flops": work[j][0], "distinct_propagators": distinct[j]}
    j = max(roof, key=lambda k: roof[k]["pass_us"]) if roof else None
    if j is not None:
        r = roof[j]
        hbm = r["algorithmic_bytes"] / HBM_PEAK >= r["algorithmic_flops"] / PEAK[prec]
        top = {"bound": "hbm" if hbm else "mfma", "achieved": r["GB/s"] if hbm else r["TFLOP/s"],
               "peak": HBM_PEAK / 1e9 if hbm else PEAK[prec] / 1e12, "unit": "GB/s" if hbm else "TFLOP/s",
               "frac": r["hbm_frac"] if hbm else r["mfma_frac"], "traffic": None,
               "kernel": f"grouped fibre pass, {j} ({prec}), all systems"}
    else:
        top = None
    out = {"metric": METRIC + " (batched systems)", "value": coeffs * args.steps / (ms_batch * 1e-3),
           "unit": "coeff*steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_batch / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": DTYPE[prec], "data": "synthetic",
           "config": {"workload": f"batch_{args.batch_1d}x1d_{args.batch_2d}x2d_W16_kappa{args.kappa:g}",
                      "systems": len(items), "total_coefficients": coeffs,
                      "N_range": [min(it[0].N for it in items), max(it[0].N for it in items)],
                      "tiles": {"layer1": B.tuning(1)[:2], "layer2": B.tuning(2)[:2]},
                      "launch_mode": {"layer1": B.tuning(1)[3], "layer2": B.tuning(2)[3]}},
           "sequential_value": coeffs * args.steps / (ms_seq * 1e-3), "sequential_ms_per_step": ms_seq / args.steps,
           "precompute_s": pre, "roofline": top, "passes": roof}
    print(json.dumps(out))
    B.destroy()
    for S, P, st in items:
        st.destroy()
        P.destroy()
        S.destroy()


def learned_workload(args):
    """Learned importance-sampling proposal on the twisted bilayer (triangular lattices at
    +-2.5 deg, Ec = 6500: N = 398821, 889 + 889 fibres), stochastic Strang layer splitting with
    tau = 5e-3 to T = 1 (200 steps), precision = first of `--paths`.  kappa = 1: the kinetic part
    is the exact phase and the sampled fibre flows are potential-only, so every fibre increment
    (P_f - I) c_f is O(tau |V|) and importance weights above 1 do not blow the estimate up (with
    kappa = 0, |P_f - I| reaches 2 on high-energy components and the weighted estimates diverge).

    Training: `--learn-traj` plain trajectories (k0 area-uniform in |k0| <= 5, seed 0, sigma = 3),
    features and optimal-proposal targets of both sub-steps every 20 steps, `--train-iters`
    full-batch Adam steps on the GPU.  Evaluation: 8 held-out wavepackets (seed 1) x 16
    realisations each (W = 128): the learned proposal with `--learn-p` draws per sub-step, the
    uniform proposal at the same expected propagator work, and the deterministic step as the
    reference (L2 error after T, variance of energy and mass over realisations).
    """
    import math
    import torch
    from paper_2103_14897_amd import proposal

    prec = args.paths.split(",")[0]
    p = args.learn_p
    eps = 0.05
    spec = wl.twisted_system(6500.0)
    tau, K = 5e-3, args.learn_steps
    stream = torch.cuda.current_stream()
    S = lsx.System.from_spec(spec)
    mn = S.index()
    nin = spec.d + 3
    t0 = time.perf_counter()
    P = lsx.Plan(S, tau, "strang", 1.0, prec, stream)
    pre = time.perf_counter() - t0
    Ls = {l: np.diff(S.fibres(l)[0]).astype(np.float64) for l in (1, 2)}
    # ---- training data from plain trajectories
    Wt = args.learn_traj
    st = lsx.State(P, Wt)
    sm = lsx.Sampler(st, p, p, eps)
    st.upload(wl.gaussian_state(spec, mn, wl.draw_k0(Wt, 2, seed=0, kmax=5.0), 3.0), stream)
    t0 = time.perf_counter()
    X, b, gptr = proposal.collect(sm, st, K, 20, stream)
    torch.cuda.synchronize()
    t_collect = time.perf_counter() - t0
    sm.destroy()
    st.destroy()
    M = int(X.shape[0])
    net = lsx.Mlp(nin)
    net.set(wl.mlp_init(nin, 64, seed=0))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    log = proposal.train(net, X, b, gptr, args.train_iters, 3e-3, eps, log_every=max(1, args.train_iters // 6),
                         stream=stream)
    e1.record(stream)
    e1.synchronize()
    ms_train = e0.elapsed_time(e1) / args.train_iters
    # flops per row of one train step: forward 2 (nin H + H^2 + H); backward recomputes the
    # forward and adds W2 delta2, the W2 and W1 outer products (2 H^2 each) and 2 nin H
    H = 64
    fl_row = 2 * (nin * H + H * H + H) + 2 * (nin * H + H * H) + 2 * H * H + 2 * H * H + 2 * nin * H
    train_tf = fl_row * M / (ms_train * 1e-3) / 1e12
    del X, b, gptr
    # ---- held-out evaluation: 8 wavepackets x 16 realisations
    nw, nr = 8, 16
    W = nw * nr
    k0 = np.repeat(wl.draw_k0(nw, 2, seed=1, kmax=5.0), nr, axis=0)
    c0 = wl.gaussian_state(spec, mn, k0, 3.0)
    st = lsx.State(P, W)
    sm = lsx.Sampler(st, p, p, eps)
    st.upload(c0, stream)
    obj, cost_l, cost_u = {}, [], []
    for layer, half in proposal.substep_layers("strang"):
        nf = S.nfibres[layer]
        Xv = torch.empty((W, nf, nin), dtype=torch.float32, device="cuda")
        bv = torch.empty((W, nf), dtype=torch.float64, device="cuda")
        sm.features(layer, Xv, stream)
        sm.increments(layer, half, bv, stream)
        obj[f"layer{layer}"] = {"uniform": proposal.objective(None, Xv.reshape(-1, nin), bv.reshape(-1), nf, eps),
                                "learned": proposal.objective(net, Xv.reshape(-1, nin), bv.reshape(-1), nf, eps)}
        z = torch.empty(W * nf, dtype=torch.float32, device="cuda")
        net.forward(Xv.reshape(-1, nin), W * nf, z, stream)
        zz = z.reshape(W, nf).double().cpu().numpy()
        q = np.exp(zz - zz.max(axis=1, keepdims=True))
        q = (1 - eps) * q / q.sum(axis=1, keepdims=True) + eps / nf
        cost_l.append(float((q * Ls[layer][None, :] ** 2).sum(axis=1).mean()))
        cost_u.append(float((Ls[layer] ** 2).mean()))
    # expected propagator work per draw (sum of L^2 weighted by q) at the initial states
    pu = int(math.ceil(p * sum(cost_l) / sum(cost_u)))
    sm.destroy()
    runs = {}
    ref = lsx.State(P, W)
    ref.upload(c0, stream)
    e0.record(stream)
    ref.step(K, stream)
    e1.record(stream)
    e1.synchronize()
    runs["deterministic"] = {"ms_per_step": e0.elapsed_time(e1) / K}
    det = ref.download(stream)
    obs_det = ref.observables(lsx.OBS_MASS | lsx.OBS_ENERGY, stream)
    ref.destroy()
    for name, pp, mlp in (("learned", p, net), ("uniform_equal_cost", pu, None), ("uniform_equal_p", p, None)):
        smr = lsx.Sampler(st, pp, pp, eps)
        smr.set_mlp(mlp)
        u = torch.as_tensor(wl.uniforms((K, 3, W, pp), seed=7), device="cuda")
        st.upload(c0, stream)
        torch.cuda.synchronize()
        e0.record(stream)
        smr.ss_step(u, K, stream)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / K
        x = st.download(stream)
        obs = st.observables(lsx.OBS_MASS | lsx.OBS_ENERGY, stream)
        err = np.linalg.norm(x - det, axis=0)
        runs[name] = {"p": pp, "ms_per_step": ms,
                      "l2_error_mean": float(err.mean()), "l2_error_median": float(np.median(err)),
                      "energy_var_mean": float(obs["energy"].reshape(nw, nr).var(axis=1).mean()),
                      "energy_bias_mean": float(np.abs(obs["energy"].reshape(nw, nr).mean(axis=1)
                                                       - obs_det["energy"].reshape(nw, nr)[:, 0]).mean()),
                      "mass_var_mean": float(obs["mass"].reshape(nw, nr).var(axis=1).mean())}
        smr.set_mlp(None)
        smr.destroy()
        del u
    st.destroy()
    out = {"metric": "coeff·steps/s of learned stochastic layer splitting; L2 error and observable variance "
                     "vs uniform sampling at equal cost",
           "value": S.N * W / (runs["learned"]["ms_per_step"] * 1e-3), "unit": "coeff*steps/s", "n_gpus": 1,
           "steps": K, "warmup": 0, "ms_per_step": runs["learned"]["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[prec] + " (network f32)", "data": "synthetic",
           "config": {"workload": "twisted_tri_pm2.5deg_Ec6500_kappa1_stochastic_strang_tau5e-3_learned_proposal",
                      "N": S.N, "fibres": [S.nfibres[1], S.nfibres[2]], "p": p, "eps": eps,
                      "train_trajectories": Wt, "eval_columns": f"{nw} wavepackets x {nr} realisations"},
           "training": {"rows": M, "iters": args.train_iters, "ms_per_iter": ms_train, "collect_s": t_collect,
                        "objective_log": log, "plan_precompute_s": pre},
           "heldout_objective": obj,
           "expected_work_per_draw": {"learned": sum(cost_l) / 2, "uniform": sum(cost_u) / 2},
           "runs": runs,
           "roofline": {"bound": "mfma", "achieved": train_tf, "peak": 157.3, "unit": "TFLOP/s",
                        "frac": train_tf / 157.3, "traffic": None,
                        "kernel": "proposal network train step (forward + objective + backward + Adam); "
                                  "hidden-layer products on FP32 MFMA, first layer and tanh on the VALU"}}
    print(json.dumps(out))
    net.destroy()
    P.destroy()
    S.destroy()


def si_workload(args):
    """Semi-implicit (Alg. 1) and random batch (Alg. 4, 1/10 of the fibres per layer) steps on the
    twisted bilayer (Ec = 6500, N = 398821, W = 128, tau = 5e-3): one neighbour-stencil kernel per
    step, HBM-bound.  The plan is built with kappa = 1 (these steps use only |K|^2 and the stencil)."""
    import torch

    w = wl.twisted()
    S = lsx.System.from_spec(w.spec)
    P = lsx.Plan(S, w.tau, "strang", 1.0, "fp64")
    W, N = w.W, S.N
    c0 = w.initial_state(S.index())
    st = lsx.State(P, W)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    st.upload(c0, stream)
    st.si_step(args.warmup, stream)
    e0.record(stream)
    st.si_step(args.steps, stream)
    e1.record(stream)
    e1.synchronize()
    res["alg1"] = {"ms_per_step": e0.elapsed_time(e1) / args.steps}
    st.upload(c0, stream)
    st.si_step(w.nsteps, stream)
    res["alg1"]["mass_after_T"] = float(st.observables(lsx.OBS_MASS, stream)["mass"].mean())
    p1, p2 = max(1, S.nfibres[1] // 10), max(1, S.nfibres[2] // 10)
    sm = lsx.Sampler(st, p1, p2)
    u = torch.as_tensor(wl.uniforms((args.steps, 2, W, max(p1, p2)), seed=3), device="cuda")
    st.upload(c0, stream)
    e0.record(stream)
    sm.rb_step(u, args.steps, stream)
    e1.record(stream)
    e1.synchronize()
    res["alg4"] = {"ms_per_step": e0.elapsed_time(e1) / args.steps, "p": [p1, p2]}
    sm.destroy()
    nv = len(w.spec.pot1) + len(w.spec.pot2)
    # algorithmic bytes of one stencil launch: read and write the state, |K|^2 and the stencil
    # table (neighbour rows are read again from cache, not from HBM)
    nbytes = 2.0 * N * W * 16 + 8.0 * N + 4.0 * nv * N
    t = res["alg1"]["ms_per_step"] * 1e-3
    out = {"metric": "coeff·steps/s of the semi-implicit step (Alg. 1); random batch (Alg. 4) beside it",
           "value": N * W / t, "unit": "coeff*steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": res["alg1"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "twisted_tri_pm2.5deg_Ec6500_W128_semi_implicit_tau5e-3", "N": N, "W": W},
           "runs": res,
           "roofline": {"bound": "hbm", "achieved": nbytes / t / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                        "frac": nbytes / t / HBM_PEAK, "traffic": None, "kernel": "k_si_step (Alg. 1)",
                        "algorithmic_bytes": nbytes}}
    print(json.dumps(out))
    st.destroy()
    P.destroy()
    S.destroy()


def trilayer_workload(args):
    """Three layers: the twisted triangular trilayer (layers at -2.5, 0, +2.5 deg, first-shell
    potentials 1.0, 0.5, 0.7), ball cutoff Ec = 1000 (N = 415135, 9061 fibres per layer of length
    up to 139), 128 random unit wavepackets (seed 0), tau = 5e-3, kappa = 0.  Each path runs
    50 steps from the same state for the error against FP64, then the timed steps; every
    layer's pass is timed on its own (slot tau for layers 1 and 3, tau/2 for layer 2 of the
    Strang plan)."""
    spec = wl.twisted_layers(1000.0)
    S = lsx.System.layers(spec.d, spec.As, spec.Ec, spec.cutoff, spec.pots)
    slot = {"strang": {1: 0, 2: 1, 3: 0}, "lie": {1: 0, 2: 0, 3: 0}, "yoshida4": {1: 0, 2: 0, 3: 0}}[args.scheme]
    return layered_bench(args, S, 128, 5e-3, slot, "three-layer splitting",
                         f"twisted_trilayer_m2.5_0_p2.5deg_Ec1000_W128_{args.scheme}_tau5e-3")


def example3_workload(args):
    """Example 3 of Sec. 5 (x incommensurate, y periodic for both layers): V = cos^2(beta x)
    cos^2(pi y/2) + 2 cos^2(x) cos^2(pi y/2), beta = golden ratio - 1, lifted by (m, p, n) with
    layer 1 on (m, p) and layer 2 on (p, n); cutoff Ec = 1000 (N = 74037; 45 + 73 fibres of
    length up to 2117 and 1305), 128 random unit wavepackets (seed 0), tau = 5e-3, kappa = 0.
    Same measurements as the trilayer mode."""
    spec = wl.example3_system(1000.0)
    S = lsx.System.blocks(spec.Rs, spec.groups, spec.Ec, spec.layers, spec.pots)
    slot = {"strang": {1: 0, 2: 0}, "lie": {1: 0, 2: 0}, "yoshida4": {1: 0, 2: 0}}[args.scheme]
    return layered_bench(args, S, 128, 5e-3, slot, "Example-3 layer splitting",
                         f"example3_quasi1d_Ec1000_W128_{args.scheme}_tau5e-3")


def layered_bench(args, S, W, tau, slot, what, workload):
    import torch

    N = S.N
    layers = sorted(slot)
    c0 = wl.random_state(N, W, seed=0)
    sumL2 = {j: int(np.sum(np.diff(S.fibres(j)[0]).astype(np.int64) ** 2)) for j in layers}
    stream = torch.cuda.current_stream()
    res, finals = {}, {}
    for path in args.paths.split(","):
        P = lsx.Plan(S, tau, args.scheme, args.kappa, path, stream)
        st = lsx.State(P, W)
        st.upload(c0, stream)
        st.step(50, stream)
        finals[path] = st.download(stream)
        st.upload(c0, stream)
        st.step(args.warmup, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        st.step(args.steps, stream)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        passes = {}
        for j in layers:
            st.fibre_pass(j, slot[j], max(args.kernel_reps // 4, 1), stream)
            e0.record(stream)
            st.fibre_pass(j, slot[j], args.kernel_reps, stream)
            e1.record(stream)
            e1.synchronize()
            passes[j] = e0.elapsed_time(e1) * 1e3 / args.kernel_reps
        res[path] = {"coeff_steps_per_s": N * W * args.steps / (ms * 1e-3), "ms_per_step": ms / args.steps,
                     "pass_us": passes, "tiles": {j: st.tuning(j)[:2] + (st.prefetch(j),) for j in layers},
                     "nontemporal_stores": st.store_mode()[0],
                     "band_kept": {j: P.band(j)[1] / max(P.band(j)[2], 1) for j in layers},
                     "_kept": {j: P.band(j, stored=True) for j in layers}}
        st.destroy()
        P.destroy()
    ref = finals.get("fp64")
    for path in res:
        res[path]["rel_l2_vs_fp64_50_steps"] = None if ref is None else float(
            (np.linalg.norm(finals[path] - ref, axis=0) / np.linalg.norm(ref, axis=0)).max())
    ok = [p for p in res if p == "fp64" or ref is None or res[p]["rel_l2_vs_fp64_50_steps"] <= 1e-6]
    best = max(ok, key=lambda p: res[p]["coeff_steps_per_s"])
    r = res[best]
    j = max(r["pass_us"], key=lambda k: r["pass_us"][k])  # dominant pass
    _, kept, _, skept, srows = r["_kept"][j]  # band-limited products (lsx_plan_band)
    flops = 8.0 * W * kept
    nbytes = 2.0 * N * W * 16 + PROP_BYTES[best] * skept + (16.0 * srows if best != "fp64" else 0.0)
    t = r["pass_us"][j] * 1e-6
    bound = "mfma" if flops / PEAK[best] >= nbytes / HBM_PEAK else "hbm"
    if bound == "mfma":
        roof = {"bound": "mfma", "achieved": flops / t / 1e12, "peak": PEAK[best] / 1e12, "unit": "TFLOP/s",
                "frac": flops / t / PEAK[best]}
    else:
        roof = {"bound": "hbm", "achieved": nbytes / t / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": nbytes / t / HBM_PEAK}
    for q in res.values():
        q.pop("_kept", None)
    roof.update({"traffic": None, "kernel": f"fibre pass, layer {j} ({best})", "algorithmic_flops": flops,
                 "algorithmic_bytes": nbytes, "dense_flops": 8.0 * W * sumL2[j],
                 "other_roof_frac": (nbytes / t / HBM_PEAK) if bound == "mfma" else (flops / t / PEAK[best])})
    out = {"metric": f"coeff·steps/s of {what}; % HBM/MFMA peak of the dominant pass",
           "value": r["coeff_steps_per_s"], "unit": "coeff*steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": DTYPE[best], "data": "synthetic",
           "config": {"workload": workload, "N": N,
                      "W": W, "fibres": [S.nfibres[j] for j in layers], "path": best,
                      "kappa": args.kappa, "scheme": args.scheme},
           "roofline": roof, "paths": res}
    print(json.dumps(out))
    S.destroy()


def time_paths(S, w, c0, paths, scheme, kappa, steps, warmup, reps, stream):
    """Per precision path: plan precompute, an accuracy run to T, `warmup` untimed then `steps`
    timed steps (HIP events on `stream`, the stream every kernel is launched on), and `reps`
    back-to-back launches of each layer's pass (and of the phase when kappa > 0).  Returns the
    per-path results (with the max relative L2 against the FP64 path after T) and the states
    after T."""
    import torch

    N, W = S.N, w.W
    res = {}
    finals = {}
    for path in paths:
        t0 = time.perf_counter()
        P = lsx.Plan(S, w.tau, scheme, kappa, path, stream)
        pre = time.perf_counter() - t0
        st = lsx.State(P, W)
        # accuracy run to T
        st.upload(c0, stream)
        st.step(w.nsteps, stream)
        finals[path] = st.download(stream)
        moved = float((np.linalg.norm(finals[path] - c0, axis=0) / np.linalg.norm(c0, axis=0)).max())
        # timed run
        st.upload(c0, stream)
        st.step(warmup, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        st.step(steps, stream)
        e1.record(stream)
        e1.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1)
        # each layer's pass, back-to-back launches on the same stream, after an untimed quarter
        # of them (the GPU idles during the synchronisation before)
        torch.cuda.synchronize()
        k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        st.fibre_pass(2, 0, max(reps // 4, 1), stream)
        k0.record(stream)
        st.fibre_pass(2, 0, reps, stream)
        k1.record(stream)
        k1.synchronize()
        kus = k0.elapsed_time(k1) * 1e3 / reps
        st.fibre_pass(1, 0, max(reps // 4, 1), stream)
        k0.record(stream)
        st.fibre_pass(1, 0, reps, stream)
        k1.record(stream)
        k1.synchronize()
        kus1 = k0.elapsed_time(k1) * 1e3 / reps
        phase_us = None
        if kappa != 0.0:
            k0.record(stream)
            for _ in range(reps):
                st.phase(1, stream)
            k1.record(stream)
            k1.synchronize()
            phase_us = k0.elapsed_time(k1) * 1e3 / reps
        band = {j: P.band(j, stored=True) for j in (1, 2)}
        res[path] = {"coeff_steps_per_s": N * W * steps / (ms * 1e-3), "ms_per_step": ms / steps,
                     "wall_ms": wall * 1e3, "precompute_s": pre, "layer2_pass_us": kus, "layer1_pass_us": kus1,
                     "tiles": {"layer1": st.tuning(1)[:2] + (st.prefetch(1),),
                               "layer2": st.tuning(2)[:2] + (st.prefetch(2),)},
                     "nontemporal_stores": st.store_mode()[0], "rel_change_after_T": moved,
                     "band_tol": band[1][0],
                     "band_kept": {f"layer{j}": band[j][1] / max(band[j][2], 1) for j in (1, 2)},
                     "_kept": {j: band[j][1] for j in (1, 2)},
                     "_stored": {j: band[j][3:] for j in (1, 2)}}
        if phase_us is not None:
            res[path]["phase_us"] = phase_us
            res[path]["phase_GBps"] = (2.0 * N * W * 16 + 16.0 * N) / (phase_us * 1e-6) / 1e9
        print(f"[bench] N={N} W={W} {path}: precompute {pre:.2f} s, {ms / steps * 1e3:.1f} us/step, "
              f"relative change after T {moved:.3f}", file=sys.stderr, flush=True)
        st.destroy()
        P.destroy()
    ref = finals.get("fp64")
    for path in res:
        res[path]["rel_l2_vs_fp64_after_T"] = (
            float((np.linalg.norm(finals[path] - ref, axis=0) / np.linalg.norm(ref, axis=0)).max())
            if ref is not None else None)
    return res, finals


def config3_summary(args, stream):
    """The MFMA-bound twisted bilayer (triangular lattices at +-2.5 deg, Ec = 6500, N = 398821,
    W = 128, Strang tau = 5e-3 to T = 1) on every path: ms/step, coeff*steps/s, max relative L2
    against the FP64 path after T (200 steps), and each layer pass against its path's MFMA peak
    (8 W flops per complex multiply-add the band-limited pass performs; the dense count 8 W
    sum L^2 beside it)."""
    w = wl.twisted()
    S = lsx.System.from_spec(w.spec)
    c0 = w.initial_state(S.index())
    sumL2 = {j: int(np.sum(np.diff(S.fibres(j)[0]).astype(np.int64) ** 2)) for j in (1, 2)}
    res, finals = time_paths(S, w, c0, args.paths.split(","), "strang", 0.0, args.config3_steps, 2, 4, stream)
    del finals
    out = {"workload": "twisted_tri_pm2.5deg_Ec6500_W128_strang_tau5e-3", "N": S.N, "W": w.W,
           "steps_to_T": w.nsteps, "timed_steps": args.config3_steps, "paths": {}}
    for path, r in res.items():
        q = {k: r[k] for k in ("ms_per_step", "coeff_steps_per_s", "rel_l2_vs_fp64_after_T", "rel_change_after_T",
                               "precompute_s",
                               "layer1_pass_us", "layer2_pass_us", "tiles", "nontemporal_stores", "band_tol",
                               "band_kept")}
        for j in (1, 2):
            t = r[f"layer{j}_pass_us"] * 1e-6
            tf = 8.0 * w.W * r["_kept"][j] / t
            q[f"layer{j}_pass_TFLOPs"] = tf / 1e12
            q[f"layer{j}_pass_mfma_frac"] = tf / PEAK[path]
            q[f"layer{j}_pass_dense_equivalent_TFLOPs"] = 8.0 * w.W * sumL2[j] / t / 1e12
        out["paths"][path] = q
    S.destroy()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--paths", default="fp64,mix_fp32,mix_bf16x3")
    ap.add_argument("--kernel-reps", type=int, default=400)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-config3", action="store_true",
                    help="chain workload: leave out the twisted-bilayer summary added to the line")
    ap.add_argument("--config3-steps", type=int, default=20)
    ap.add_argument("--calib-mib", type=int, default=64)
    ap.add_argument("--batch-1d", type=int, default=240)
    ap.add_argument("--batch-2d", type=int, default=16)
    ap.add_argument("--learn-traj", type=int, default=200)
    ap.add_argument("--learn-p", type=int, default=16)
    ap.add_argument("--train-iters", type=int, default=300)
    ap.add_argument("--learn-steps", type=int, default=200, help="learned mode: evaluation steps (T = steps tau)")
    ap.add_argument("--workload", default="chain",
                    choices=["chain", "twisted", "twisted1", "tiny", "batch", "learned", "si", "trilayer",
                             "example3"],
                    help="chain: the metric's workload (default); the others are extra measurements")
    ap.add_argument("--kappa", type=float, default=0.0)
    ap.add_argument("--chain-ec", type=float, default=2.0e4,
                    help="chain workload cutoff (9.71e4 gives the count-matched N = 25019)")
    ap.add_argument("--scheme", default="strang", choices=["strang", "lie", "yoshida4", "strang_cn", "lie_be"],
                    help="composition of the timed steps (the metric is quoted on strang)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the lifted step shards by wavepacket with no "
              "communication, so the N-GPU figure is N x the one-GPU figure; run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    if args.workload == "batch":
        return batch_workload(args)
    if args.workload == "learned":
        return learned_workload(args)
    if args.workload == "si":
        return si_workload(args)
    if args.workload == "trilayer":
        return trilayer_workload(args)
    if args.workload == "example3":
        return example3_workload(args)
    w = {"chain": lambda: wl.chain(Ec=args.chain_ec), "twisted": wl.twisted, "twisted1": lambda: wl.twisted(W=1),
         "tiny": wl.tiny_chain}[args.workload]()
    S = lsx.System.from_spec(w.spec)
    mn = S.index()
    c0 = w.initial_state(mn)
    N, W = S.N, w.W
    ptr2, _ = S.fibres(2)
    ptr1, _ = S.fibres(1)
    sumL2 = {1: int(np.sum(np.diff(ptr1).astype(np.int64) ** 2)), 2: int(np.sum(np.diff(ptr2).astype(np.int64) ** 2))}
    stream = torch.cuda.current_stream()
    # calibration copy of known size (64 MiB read + 64 MiB written), outside any timed
    # region: its FETCH_SIZE / WRITE_SIZE counters scale the pass counters to bytes
    calib_a = torch.ones(args.calib_mib << 17, dtype=torch.float64, device="cuda")
    calib_b = torch.empty_like(calib_a)
    calib_b.copy_(calib_a)
    torch.cuda.synchronize()
    del calib_a, calib_b
    res, finals = time_paths(S, w, c0, args.paths.split(","), args.scheme, args.kappa, args.steps, args.warmup,
                             args.kernel_reps, stream)
    ref = finals.get("fp64")
    # without the FP64 path there is no reference: every path is eligible (its error is null)
    ok = [p for p in res if p == "fp64" or ref is None or (res[p]["rel_l2_vs_fp64_after_T"] is not None
                                                           and res[p]["rel_l2_vs_fp64_after_T"] <= 1e-6)]
    best = max(ok, key=lambda p: res[p]["coeff_steps_per_s"])
    r = res[best]
    # dominant kernel: the layer-2 fibre pass.  Algorithmic work per launch: the band-limited
    # complex products, 8 W flops per propagator entry inside the band (lsx_plan_band; the
    # dense count would be sum L^2 entries); bytes: read + write the state (2 N W 16) plus the
    # band entries of the stored propagators, each read once (fibres that share a propagator
    # through a point symmetry count it once), and on the mixed paths their FP64 diagonals.
    kept = r["_kept"][2]
    skept, srows = r["_stored"][2]
    flops = 8.0 * W * kept
    nbytes = 2.0 * N * W * 16 + PROP_BYTES[best] * skept + (16.0 * srows if best != "fp64" else 0.0)
    t = r["layer2_pass_us"] * 1e-6
    bound = "mfma" if flops / PEAK[best] >= nbytes / HBM_PEAK else "hbm"
    if bound == "mfma":
        roof = {"bound": "mfma", "achieved": flops / t / 1e12, "peak": PEAK[best] / 1e12, "unit": "TFLOP/s",
                "frac": flops / t / PEAK[best]}
    else:
        roof = {"bound": "hbm", "achieved": nbytes / t / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": nbytes / t / HBM_PEAK}
    ec_tag = ("%.3g" % args.chain_ec).replace("e+0", "e").replace("e+", "e")
    counted = args.workload == "chain" and args.kappa == 0.0 and args.chain_ec == 2.0e4
    roof.update({"traffic": measured_traffic(best) if counted else None,
                 "kernel": f"fibre pass, layer 2 ({best})",
                 "algorithmic_flops": flops, "algorithmic_bytes": nbytes,
                 "dense_flops": 8.0 * W * sumL2[2],
                 "dense_bytes": 2.0 * N * W * 16 + PROP_BYTES[best] * sumL2[2] + (16.0 * N if best != "fp64" else 0.0),
                 "other_roof_frac": (nbytes / t / HBM_PEAK) if bound == "mfma" else (flops / t / PEAK[best])})
    for q in res.values():
        q.pop("_kept", None)
        q.pop("_stored", None)
    out = {
        "metric": METRIC,
        "value": r["coeff_steps_per_s"],
        "unit": "coeff*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[best],
        "data": "synthetic",
        "config": {"workload": {"chain": f"chain1d_golden_Ec{ec_tag}_W64_{args.scheme}_tau1e-3",
                                "twisted": f"twisted_tri_pm2.5deg_Ec6500_W128_{args.scheme}_tau5e-3",
                                "twisted1": f"twisted_tri_pm2.5deg_Ec6500_W1_{args.scheme}_tau5e-3",
                                "tiny": f"chain1d_golden_Ec200_W1_{args.scheme}_tau1e-2"}[args.workload],
                   "N": N, "W": W, "fibres": [S.nfibres[1], S.nfibres[2]], "path": best, "kappa": args.kappa,
                   "scheme": args.scheme},
        "roofline": roof,
        "paths": res,
    }
    if counted and not args.no_config3:
        out["config3"] = config3_summary(args, stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w.spec, c0, w.tau)
    print(json.dumps(out))
    S.destroy()


if __name__ == "__main__":
    main()
