"""The batched MaxCut workload: 512 uneven instances, R = 32 replicas each.

Workload: N log-uniform in [1000, 50000] (seeds 50000 + b), even b random
3-regular, odd b G(n, 5n), +/-1 weights, h0 ~ N(0, 0.01^2) per instance
(seed 1000000 + instance seed), linear beta 0.01 -> 5, Adam lr 0.1.

Two measurements:

* throughput: the block-diagonal union of the 512 instances stepped by one
  launch per step (bfloat16 marginal copy, float32 fields and Adam state,
  per-replica energies every step, anytime read-out every 25 steps), K steps
  in one captured HIP graph from device-resident inputs;
* time to a target cut.  Plain FEM is float32, one solver per instance, its
  T_plain-step anneal captured as a HIP graph before the clock starts and h0
  already on the device; C_plain(b) is the best replica's cut of instance b
  and the target of b is C_plain(b) - 0.001 |C_plain(b)|.  The variants run
  on the union in one launch per step (HIP-graph chunks of K steps, anytime
  read-out every K steps): batched float32, batched bfloat16, and batched
  bfloat16 with the learned warm start (the first T_early steps of the plain
  bfloat16 anneal, the network's proposal h = alpha z for every replica, then
  a second anneal of T_warm steps with beta from beta_start to 5); the
  ablation continues from the fields themselves instead of the proposal.
  Each variant reports two times: until every instance's best cut reaches its
  own target, and until the sum over instances of the best cuts reaches the
  sum of the targets; network inference is inside the clock, training is not.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

from paper_2412_09285_amd import fem
from paper_2412_09285_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PARAMS = os.path.join(HERE, "data", "mpnn_maxcut.bin")
R_BATCH = 32


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def instances(n_inst=512):
    return [W.batch_instance(b) for b in range(n_inst)]


def h0_for(g, R):
    return W.initial_fields(g.n, R, seed=1_000_000 + g.meta["seed"])


class Batch:
    """The instances, their problems (each alone and as one union) and their
    initial fields on the device."""

    def __init__(self, graphs, R=R_BATCH):
        import torch

        self.graphs, self.R = graphs, R
        self.parts = [fem.Problem.maxcut(g.n, g.u, g.v, g.w) for g in graphs]
        self.union = fem.Problem.batch(self.parts)
        self.h0_parts = [torch.from_numpy(h0_for(g, R)).cuda() for g in graphs]
        self.h0 = torch.cat(self.h0_parts)
        self.n = sum(g.n for g in graphs)
        self.nnz = sum(g.nnz for g in graphs)


def throughput(b: Batch, K, Wm, stream, dtype=fem.BF16, eval_every=25, tune=True, profile_steps=50):
    """Updates/s over K graph-captured steps of the union, and the step
    kernel's average duration from HIP events on the solver's stream."""
    import torch

    T = max(K, Wm, 1)
    s = fem.Solver(b.union, fem.default_params(replicas=b.R, steps=T, energy_every=1, marginal_dtype=dtype,
                                               eval_every=min(eval_every, K)), stream=stream)
    s.set_fields(b.h0)
    tile = s.tune(trial_steps=5, use_cache=True) if tune else s.tile()
    s.set_fields(b.h0)
    s.step(min(Wm, T))
    s.sync()
    s.set_fields(b.h0)
    s.capture(K)
    s.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run_until(K)
    s.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    U = s.energies()[0]
    best = s.anytime_best().max(axis=1)
    s.set_fields(b.h0)
    s.profile(True)
    s.step(min(profile_steps, T))
    kern_ms, n_k = s.profile_result()
    s.profile(False)
    s.close()
    return dict(seconds=dt, updates_per_s=b.nnz * b.R * K / dt, tile=tile, kernel_ms=kern_ms, kernel_launches=n_k,
                U_mean=float(np.mean(U)), best_sum=float(best.sum()))


def gaps(best, plain):
    g = (best - plain) / np.maximum(np.abs(plain), 1)
    return {"min": float(g.min()), "median": float(np.median(g)), "max": float(g.max()),
            "instances_at_target": int(np.sum(best >= plain - 0.001 * np.abs(plain)))}


def plain_per_instance(b: Batch, T, stream):
    """Plain float32 FEM, one solver per instance: every anneal captured as a
    HIP graph before the clock, h0 on the device; timed: for each instance
    set the fields, launch its graph, read its best replica."""
    import torch

    solvers = [fem.Solver(p, fem.default_params(replicas=b.R, steps=T, energy_every=0), stream=stream)
               for p in b.parts]
    t_cap = time.perf_counter()
    for s, h0 in zip(solvers, b.h0_parts):
        s.set_fields(h0)
        s.capture(T)
    torch.cuda.synchronize()
    t_cap = time.perf_counter() - t_cap
    vals = []
    t0 = time.perf_counter()
    for s, h0 in zip(solvers, b.h0_parts):
        s.set_fields(h0)
        s.run_until(T)
        _, val, _ = s.best()
        vals.append(int(val[0]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for s in solvers:
        s.close()
    return np.array(vals, dtype=np.float64), wall, t_cap


class Clock:
    """Time to target under both criteria, from the per-instance best so far."""

    def __init__(self, plain):
        self.target = plain - 0.001 * np.abs(plain)
        self.target_sum = float(self.target.sum())
        self.t0 = time.perf_counter()
        self.t_all = self.t_sum = None
        self.steps_all = self.steps_sum = None
        self.best_at_all = None

    def check(self, best, steps):
        now = time.perf_counter() - self.t0
        if self.t_sum is None and float(best.sum()) >= self.target_sum:
            self.t_sum, self.steps_sum = now, steps
        if self.t_all is None and bool(np.all(best >= self.target)):
            self.t_all, self.steps_all, self.best_at_all = now, steps, best.copy()
        return self.t_all is not None and self.t_sum is not None


def _chunks(T, K):
    return [(a, min(T, a + K)) for a in range(0, T, K)]


def batched(b: Batch, plain, T, K, stream, dtype):
    """One solver on the union: chunks of K steps (captured before the
    clock), anytime best after each chunk."""
    s = fem.Solver(b.union, fem.default_params(replicas=b.R, steps=T, energy_every=0, eval_every=K,
                                               marginal_dtype=dtype), stream=stream)
    s.set_fields(b.h0)
    s.tune(trial_steps=5, use_cache=True)
    s.set_fields(b.h0)
    for (_, e) in _chunks(T, K):
        s.capture(e)
        s.run_until(e)
    s.sync()
    clk = Clock(plain)
    s.set_fields(b.h0)
    best = None
    for (_, e) in _chunks(T, K):
        s.run_until(e)
        best = s.anytime_best().max(axis=1)       # synchronises
        if clk.check(best, e):
            break
    wall = time.perf_counter() - clk.t0
    s.close()
    return clk, best, wall


def warm(b: Batch, plain, T_plain, K, stream, t_early, T_warm, beta_start, net=None, alpha=1.0, seed=5,
         dtype=fem.BF16):
    """The plain anneal's first t_early steps, then a second anneal of T_warm
    steps from the network's proposal (net=None: from the fields at
    t_early)."""
    import torch

    s1 = fem.Solver(b.union, fem.default_params(replicas=b.R, steps=T_plain, energy_every=0, eval_every=K,
                                                marginal_dtype=dtype), stream=stream)
    s2 = fem.Solver(b.union, fem.default_params(replicas=b.R, steps=T_warm, energy_every=0, eval_every=K,
                                                marginal_dtype=dtype, beta_min=beta_start), stream=stream)
    h_mid = torch.empty_like(b.h0)
    h_prop = torch.empty_like(b.h0)

    def propose():
        s1.fields(out=h_mid)
        if net is None:
            return h_mid
        # queued on the solvers' stream after the fields copy, no host wait
        net.infer(b.union, h_mid, seed=seed, alpha=alpha, out=h_prop, stream=stream)
        return h_prop

    s1.set_fields(b.h0)
    tile = s1.tune(trial_steps=5, use_cache=True)
    s2.set_tile(*tile)
    s1.set_fields(b.h0)
    for (_, e) in _chunks(t_early, K):
        s1.capture(e)
        s1.run_until(e)
    s1.sync()
    s2.set_fields(propose())
    for (_, e) in _chunks(T_warm, K):
        s2.capture(e)
        s2.run_until(e)
    s2.sync()
    torch.cuda.synchronize()
    clk = Clock(plain)
    s1.set_fields(b.h0)
    best1 = None
    done = False
    for (_, e) in _chunks(t_early, K):
        s1.run_until(e)
        best1 = s1.anytime_best().max(axis=1)
        if clk.check(best1, e):
            done = True
            break
    best = best1
    if not done:
        s2.set_fields(propose())
        for (_, e) in _chunks(T_warm, K):
            s2.run_until(e)
            best = np.maximum(best1, s2.anytime_best().max(axis=1))
            if clk.check(best, t_early + e):
                break
    wall = time.perf_counter() - clk.t0
    s1.close()
    s2.close()
    return clk, best, wall


def time_to_target(b: Batch, stream, plain_steps=1000, K=25, early_steps=100, warm_steps=300, beta_start=0.3,
                   alpha=1.0, params=DEFAULT_PARAMS):
    """The plain baseline and every variant; returns a JSON-ready dict."""
    plain, plain_wall, cap_s = plain_per_instance(b, plain_steps, stream)
    log(f"plain per instance: {plain_wall:.3f} s (graphs captured beforehand in {cap_s:.1f} s), "
        f"sum of best cuts {plain.sum():.0f}")
    res = {"plain_per_instance": {"wall_s": plain_wall, "anneal_steps": plain_steps, "sum_best": float(plain.sum()),
                                  "capture_s_untimed": cap_s}}

    def record(name, clk, best, wall, anneal):
        res[name] = {"time_to_target_all_s": clk.t_all, "steps_at_target_all": clk.steps_all,
                     "time_to_target_sum_s": clk.t_sum, "steps_at_target_sum": clk.steps_sum,
                     "ran_s": wall, "anneal_steps": anneal, "sum_best": float(best.sum()),
                     "gap_to_plain_at_end": gaps(best, plain),
                     "gap_to_plain_at_target_all": None if clk.best_at_all is None else gaps(clk.best_at_all, plain)}
        log(f"{name}: to target (every instance) {clk.t_all} s at step {clk.steps_all}; (sum) {clk.t_sum} s at "
            f"step {clk.steps_sum}; gap {res[name]['gap_to_plain_at_end']}")

    for name, dt in (("batched_f32", fem.F32), ("batched_bf16", fem.BF16)):
        record(name, *batched(b, plain, plain_steps, K, stream, dt), plain_steps)
    net = None
    if params and os.path.exists(params):
        net = fem.MPNN(np.zeros(fem.N_MPNN_PARAMS, dtype=np.float32))
        net.load(params)
    wk = dict(t_early=early_steps, T_warm=warm_steps, beta_start=beta_start)
    if net is not None:
        record("batched_bf16_warm", *warm(b, plain, plain_steps, K, stream, net=net, alpha=alpha, **wk),
               f"{early_steps} + {warm_steps}")
    record("batched_bf16_restart_without_network", *warm(b, plain, plain_steps, K, stream, net=None, **wk),
           f"{early_steps} + {warm_steps}")
    enh = res.get("batched_bf16_warm") or res["batched_bf16"]
    for crit in ("all", "sum"):
        t = enh[f"time_to_target_{crit}_s"]
        f32 = res["batched_f32"][f"time_to_target_{crit}_s"]
        res[f"speedup_{crit}"] = {"vs_plain_per_instance": plain_wall / t if t else None,
                                  "vs_batched_f32": f32 / t if (t and f32) else None}
    res["config"] = {"plain_steps": plain_steps, "early_steps": early_steps, "warm_steps": warm_steps,
                     "beta_start": beta_start, "alpha": alpha, "eval_every": K,
                     "network": os.path.basename(params) if net is not None else None}
    return res
