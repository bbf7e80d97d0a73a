"""Time to a target cut on a batch of uneven MaxCut instances.

Workload: 512 MaxCut instances, N log-uniform in [1000, 50000] (seeds 50000 +
b), even b random 3-regular, odd b G(n, 5n), +/-1 weights, R = 32 replicas.

* plain: float32 FEM per instance (one solver per instance, random h0 ~
  N(0, 0.01^2), linear beta 0.01 -> 5 over T_plain steps, Adam lr 0.1); the
  target of instance b is C_plain(b) - 0.001 |C_plain(b)| with C_plain(b) its
  best replica's cut.
* variants, all on the block-diagonal union of the 512 instances in one
  launch per step (HIP-graph chunks of K steps, anytime read-out every K
  steps): plain-batched (float32, random h0, the plain schedule); +bf16
  marginals; +warm start (network proposal h0 = alpha z, anneal from
  beta_start).  Their time to target is the wall time until the sum over
  instances of the best cut seen reaches the sum of the targets (network
  inference included for the warm start; training is separate).
"""
from __future__ import annotations

import math
import os
import sys
import time

import numpy as np

from paper_2412_09285_amd import fem
from paper_2412_09285_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PARAMS = os.path.join(HERE, "data", "mpnn_maxcut.bin")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def instances(n_inst=512):
    return [W.batch_instance(b) for b in range(n_inst)]


def h0_for(g, R):
    return W.initial_fields(g.n, R, seed=1_000_000 + g.meta["seed"])


def run_plain_per_instance(graphs, R, T, stream):
    import torch

    vals = []
    probs = [fem.Problem.maxcut(g.n, g.u, g.v, g.w) for g in graphs]
    solvers = [fem.Solver(p, fem.default_params(replicas=R, steps=T, energy_every=0), stream=stream) for p in probs]
    h0s = [h0_for(g, R) for g in graphs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, h0 in zip(solvers, h0s):
        s.set_fields(h0)
        s.step(T)
        _, val, _ = s.best()
        vals.append(int(val[0]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for s in solvers:
        s.close()
    return np.array(vals, dtype=np.int64), wall


def run_batched(graphs, R, T, K, target_sum, stream, dtype=fem.F32, beta_min=0.01, warm=None, alpha=1.0,
                n_draws=None, seed=5):
    """Returns (time to target or None, steps at target, final best sum,
    per-instance best)."""
    import torch

    parts = [fem.Problem.maxcut(g.n, g.u, g.v, g.w) for g in graphs]
    batch = fem.Problem.batch(parts)
    s = fem.Solver(batch, fem.default_params(replicas=R, steps=T, energy_every=0, eval_every=K,
                                             marginal_dtype=dtype, beta_min=beta_min), stream=stream)
    dev_h0 = torch.empty((batch.n, R), dtype=torch.float32, device="cuda")

    def initial():
        if warm is not None:
            warm.infer(batch, R=R, seed=seed, n_draws=n_draws or R, alpha=alpha, out=dev_h0)
        else:
            dev_h0.copy_(torch.from_numpy(np.concatenate([h0_for(g, R) for g in graphs])))

    chunks = [(t0, min(T, t0 + K)) for t0 in range(0, T, K)]
    # untimed pass: captures the HIP graph of every chunk (a chunk's graph is
    # keyed by its step range, so the timed pass only launches them)
    initial()
    s.set_fields(dev_h0)
    for (a, b) in chunks:
        s.capture(b)
        s.run_until(b)
    s.sync()
    torch.cuda.synchronize()
    if warm is None:
        initial()   # host-to-device copy of the random h0 stays out of the timed region
    # timed
    t_start = time.perf_counter()
    if warm is not None:
        initial()
    s.set_fields(dev_h0)
    reached, t_hit, steps_hit = False, None, None
    for (a, b) in chunks:
        s.run_until(b)
        best = s.anytime_best()        # synchronises
        tot = float(np.sum(best.max(axis=1)))
        if not reached and tot >= target_sum:
            reached, t_hit, steps_hit = True, time.perf_counter() - t_start, b
            break
    wall = time.perf_counter() - t_start
    best = s.anytime_best().max(axis=1)
    s.close()
    return (t_hit if reached else None), steps_hit, float(best.sum()), best, wall


def main_batch(args, stream):
    import torch

    R = 32
    t0 = time.time()
    graphs = instances(args.instances)
    n_nodes = sum(g.n for g in graphs)
    nnz = sum(g.nnz for g in graphs)
    log(f"{len(graphs)} instances, {n_nodes} nodes, nnz {nnz} ({time.time() - t0:.1f} s to generate)")
    plain_vals, plain_wall = run_plain_per_instance(graphs, R, args.plain_steps, stream)
    targets = plain_vals - np.floor(0.001 * np.abs(plain_vals))
    target_sum = float(np.sum(plain_vals - 0.001 * np.abs(plain_vals)))
    log(f"plain per-instance: {plain_wall:.2f} s, sum of best cuts {plain_vals.sum()}")
    res = {"plain_per_instance_s": plain_wall, "plain_sum_best": int(plain_vals.sum()),
           "target_sum": target_sum}
    K = args.eval_every
    variants = [("plain_batched_f32", dict(dtype=fem.F32, T=args.plain_steps)),
                ("batched_bf16", dict(dtype=fem.BF16, T=args.plain_steps))]
    warm = None
    if os.path.exists(args.params):
        warm = fem.MPNN(np.zeros(fem.N_MPNN_PARAMS, dtype=np.float32))
        warm.load(args.params)
        variants.append(("batched_bf16_warm", dict(dtype=fem.BF16, T=args.warm_steps, beta_min=args.beta_start,
                                                   warm=warm, alpha=args.alpha, n_draws=args.draws)))
        variants.append(("batched_bf16_cold_same_schedule",
                         dict(dtype=fem.BF16, T=args.warm_steps, beta_min=args.beta_start)))
    for name, kw in variants:
        T = kw.pop("T")
        t_hit, steps, best_sum, best, wall = run_batched(graphs, R, T, K, target_sum, stream, **kw)
        per_gap = (best - plain_vals) / np.maximum(np.abs(plain_vals), 1)
        res[name] = {"time_to_target_s": t_hit, "steps_at_target": steps, "sum_best": best_sum,
                     "ran_s": wall, "anneal_steps": T,
                     "gap_to_plain": {"min": float(per_gap.min()), "median": float(np.median(per_gap)),
                                      "max": float(per_gap.max())}}
        log(f"{name}: time to target {t_hit}, steps {steps}, sum best {best_sum:.0f}")
    tt = res.get("batched_bf16_warm", {}).get("time_to_target_s") or res["batched_bf16"]["time_to_target_s"]
    res["speedup_vs_plain"] = (plain_wall / tt) if tt else None
    res["config"] = {"instances": len(graphs), "nodes": n_nodes, "nnz": nnz, "replicas": R,
                     "plain_steps": args.plain_steps, "warm_steps": args.warm_steps, "beta_start": args.beta_start,
                     "alpha": args.alpha, "draws": args.draws, "eval_every": K}
    return res
