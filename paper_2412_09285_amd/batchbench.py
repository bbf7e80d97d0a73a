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
  marginals; +warm start: the plain bf16 anneal runs its first T_early steps,
  the network maps every replica's fields to a proposal h = alpha z, and a
  second anneal of T_warm steps continues from it with beta from beta_start
  to 5; the ablation continues from the fields themselves instead of the
  network's proposal (same schedule).  Their time to target is the wall time
  until the sum over instances of the best cut seen reaches the sum of the
  targets (network inference included; training is separate).
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


def run_batched(graphs, R, T, K, target_sum, stream, dtype=fem.F32, beta_min=0.01):
    """Returns (time to target or None, steps at target, final best sum,
    per-instance best, wall time)."""
    import torch

    parts = [fem.Problem.maxcut(g.n, g.u, g.v, g.w) for g in graphs]
    batch = fem.Problem.batch(parts)
    s = fem.Solver(batch, fem.default_params(replicas=R, steps=T, energy_every=0, eval_every=K,
                                             marginal_dtype=dtype, beta_min=beta_min), stream=stream)
    dev_h0 = torch.from_numpy(np.concatenate([h0_for(g, R) for g in graphs])).cuda()
    chunks = [(t0, min(T, t0 + K)) for t0 in range(0, T, K)]
    # untimed: the launch shape (autotuned, or cached), then the HIP graph of
    # every chunk (a chunk's graph is keyed by its step range, so the timed
    # pass only launches them)
    s.set_fields(dev_h0)
    s.tune(trial_steps=5, use_cache=True)
    s.set_fields(dev_h0)
    for (a, b) in chunks:
        s.capture(b)
        s.run_until(b)
    s.sync()
    torch.cuda.synchronize()
    # timed
    t_start = time.perf_counter()
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


def run_warm(graphs, R, K, target_sum, stream, t_early, T_plain, T_warm, beta_start, net=None, alpha=1.0, seed=5,
             dtype=fem.BF16):
    """Plain anneal for t_early steps, then a second anneal of T_warm steps
    from the network's proposal (or, with net=None, from the fields at
    t_early).  Returns (time to target or None, steps at target, final best
    sum, per-instance best, wall time)."""
    import torch

    parts = [fem.Problem.maxcut(g.n, g.u, g.v, g.w) for g in graphs]
    batch = fem.Problem.batch(parts)
    s1 = fem.Solver(batch, fem.default_params(replicas=R, steps=T_plain, energy_every=0, eval_every=K,
                                              marginal_dtype=dtype), stream=stream)
    s2 = fem.Solver(batch, fem.default_params(replicas=R, steps=T_warm, energy_every=0, eval_every=K,
                                              marginal_dtype=dtype, beta_min=beta_start), stream=stream)
    h0 = torch.from_numpy(np.concatenate([h0_for(g, R) for g in graphs])).cuda()
    h_mid = torch.empty_like(h0)
    h_prop = torch.empty_like(h0)
    c1 = [(a, min(t_early, a + K)) for a in range(0, t_early, K)]
    c2 = [(a, min(T_warm, a + K)) for a in range(0, T_warm, K)]

    def propose():
        s1.fields(out=h_mid)
        torch.cuda.current_stream().wait_stream(stream)
        torch.cuda.synchronize()
        if net is not None:
            net.infer(batch, h_mid, seed=seed, alpha=alpha, out=h_prop)
            return h_prop
        return h_mid

    # untimed: launch shapes, then every chunk graph of both solvers
    s1.set_fields(h0)
    tile = s1.tune(trial_steps=5, use_cache=True)
    s2.set_tile(*tile)
    s1.set_fields(h0)
    for (a, b) in c1:
        s1.capture(b)
        s1.run_until(b)
    s1.sync()
    s2.set_fields(propose())
    for (a, b) in c2:
        s2.capture(b)
        s2.run_until(b)
    s2.sync()
    torch.cuda.synchronize()
    # timed
    t_start = time.perf_counter()
    s1.set_fields(h0)
    hit, steps_hit = None, None
    best1 = None
    for (a, b) in c1:
        s1.run_until(b)
        best1 = s1.anytime_best().max(axis=1)
        if float(best1.sum()) >= target_sum:
            hit, steps_hit = time.perf_counter() - t_start, b
            break
    best = best1
    if hit is None:
        s2.set_fields(propose())
        for (a, b) in c2:
            s2.run_until(b)
            best = np.maximum(best1, s2.anytime_best().max(axis=1))
            if float(best.sum()) >= target_sum:
                hit, steps_hit = time.perf_counter() - t_start, t_early + b
                break
    wall = time.perf_counter() - t_start
    s1.close()
    s2.close()
    return hit, steps_hit, float(best.sum()), best, wall


def main_batch(args, stream):
    import torch

    R = 32
    t0 = time.time()
    graphs = instances(args.instances)
    n_nodes = sum(g.n for g in graphs)
    nnz = sum(g.nnz for g in graphs)
    log(f"{len(graphs)} instances, {n_nodes} nodes, nnz {nnz} ({time.time() - t0:.1f} s to generate)")
    plain_vals, plain_wall = run_plain_per_instance(graphs, R, args.plain_steps, stream)
    target_sum = float(np.sum(plain_vals - 0.001 * np.abs(plain_vals)))
    log(f"plain per-instance: {plain_wall:.2f} s, sum of best cuts {plain_vals.sum()}")
    res = {"plain_per_instance_s": plain_wall, "plain_sum_best": int(plain_vals.sum()),
           "target_sum": target_sum}
    K = args.eval_every

    def record(name, t_hit, steps, best_sum, best, wall, anneal):
        per_gap = (best - plain_vals) / np.maximum(np.abs(plain_vals), 1)
        res[name] = {"time_to_target_s": t_hit, "steps_at_target": steps, "sum_best": best_sum, "ran_s": wall,
                     "anneal_steps": anneal,
                     "gap_to_plain": {"min": float(per_gap.min()), "median": float(np.median(per_gap)),
                                      "max": float(per_gap.max())}}
        log(f"{name}: time to target {t_hit}, steps {steps}, sum best {best_sum:.0f}")

    for name, dt in (("plain_batched_f32", fem.F32), ("batched_bf16", fem.BF16)):
        t_hit, steps, best_sum, best, wall = run_batched(graphs, R, args.plain_steps, K, target_sum, stream, dtype=dt)
        record(name, t_hit, steps, best_sum, best, wall, args.plain_steps)
    warm = None
    if os.path.exists(args.params):
        warm = fem.MPNN(np.zeros(fem.N_MPNN_PARAMS, dtype=np.float32))
        warm.load(args.params)
    wk = dict(t_early=args.early_steps, T_plain=args.plain_steps, T_warm=args.warm_steps, beta_start=args.beta_start)
    if warm is not None:
        r = run_warm(graphs, R, K, target_sum, stream, net=warm, alpha=args.alpha, **wk)
        record("batched_bf16_warm", *r, f"{args.early_steps} + {args.warm_steps}")
    r = run_warm(graphs, R, K, target_sum, stream, net=None, **wk)
    record("batched_bf16_restart_without_network", *r, f"{args.early_steps} + {args.warm_steps}")
    tt = res.get("batched_bf16_warm", {}).get("time_to_target_s") or res["batched_bf16"]["time_to_target_s"]
    res["speedup_vs_plain"] = (plain_wall / tt) if tt else None
    res["config"] = {"instances": len(graphs), "nodes": n_nodes, "nnz": nnz, "replicas": R,
                     "plain_steps": args.plain_steps, "early_steps": args.early_steps, "warm_steps": args.warm_steps,
                     "beta_start": args.beta_start, "alpha": args.alpha, "eval_every": K}
    return res
