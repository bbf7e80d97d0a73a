"""Train the MaxCut warm-start network on FEM's own runs.

1. Draw the training instances of the batched MaxCut recipe (seeds 60000 + j,
   N log-uniform in [1000, 50000], even j random 3-regular, odd j G(n, 5n),
   +/-1 weights).
2. Run plain FEM on them (float32, random h0 ~ N(0, 0.01^2), R replicas, the
   linear beta anneal 0.01 -> 5 over T steps, Adam lr 0.1) as block-diagonal
   batches on the GPU; keep, for the first `keep` replicas, the fields after
   T_early steps (the network's input) and the final read-out (its label).
3. Train with fem_mpnn_train_step (hand-written forward, backward and Adam
   kernels) on minibatches of instances, each with one of its kept replicas,
   one fresh feature draw per step.
4. Save the parameters (fem_mpnn_save).

Usage: python -m paper_2412_09285_amd.train_mpnn --out PATH [--instances 2000]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2412_09285_amd import fem  # noqa: E402
from paper_2412_09285_amd import workloads as W  # noqa: E402

DEFAULT_PARAMS = os.path.join(HERE, "data", "mpnn_maxcut.bin")
TRAIN_SEED0 = 60_000


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_instances(count, seed0=TRAIN_SEED0):
    return [W.batch_instance(j, seed0=seed0) for j in range(count)]


T_PLAIN, T_EARLY = 1000, 100


def fem_runs(graphs, R=32, T=T_PLAIN, t_early=T_EARLY, keep=8, group_nodes=3_000_000, stream=None):
    """Plain FEM on block-diagonal groups of instances; returns per instance
    (fields at t_early [n][keep] float32, final read-out [n][keep] int32)."""
    out = []
    k = 0
    while k < len(graphs):
        grp = []
        nodes = 0
        while k < len(graphs) and (not grp or nodes + graphs[k].n <= group_nodes):
            grp.append(graphs[k])
            nodes += graphs[k].n
            k += 1
        parts = [fem.Problem.maxcut(g.n, g.u, g.v, g.w) for g in grp]
        batch = fem.Problem.batch(parts)
        s = fem.Solver(batch, fem.default_params(replicas=R, steps=T, energy_every=0), stream=stream)
        h0 = np.concatenate([W.initial_fields(g.n, R, seed=1_000_000 + g.meta["seed"]) for g in grp])
        s.set_fields(h0)
        s.step(t_early)
        early = s.fields()[:, :keep].copy()
        s.step(T - t_early)
        final = s.round()[:keep].T.astype(np.int32)      # [n][keep]
        offs = batch.instance_offsets()
        for b in range(len(grp)):
            out.append((early[offs[b]:offs[b + 1]], final[offs[b]:offs[b + 1]]))
        s.close()
    return out


def train(graphs, runs, epochs=12, batch_instances=40, lr=2e-3, seed=7, init_seed=1, log_every=20):
    net = fem.MPNN(W.mpnn_init_weights(init_seed))
    order_rng = np.random.default_rng(seed)
    keep = runs[0][0].shape[1]
    history = []
    step = 0
    for ep in range(epochs):
        perm = order_rng.permutation(len(graphs))
        ep_loss = []
        for s0 in range(0, len(perm), batch_instances):
            idx = perm[s0:s0 + batch_instances]
            reps = order_rng.integers(0, keep, size=len(idx))
            parts = [fem.Problem.maxcut(graphs[j].n, graphs[j].u, graphs[j].v, graphs[j].w) for j in idx]
            batch = fem.Problem.batch(parts)
            st = np.concatenate([runs[j][0][:, r] for j, r in zip(idx, reps)])
            y = np.concatenate([runs[j][1][:, r] for j, r in zip(idx, reps)])
            loss = net.train_step(batch, st, y, seed=seed + 1000 * ep, draw0=step, lr=lr)
            ep_loss.append(loss)
            step += 1
            if step % log_every == 0:
                log(f"  step {step}: loss {loss:.4f}")
        history.append(float(np.mean(ep_loss)))
        log(f"epoch {ep}: mean loss {history[-1]:.4f}")
    return net, history


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_PARAMS)
    ap.add_argument("--instances", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--label-steps", type=int, default=T_PLAIN)
    ap.add_argument("--early-steps", type=int, default=T_EARLY)
    ap.add_argument("--replicas", type=int, default=32)
    args = ap.parse_args()
    import torch

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    t0 = time.time()
    graphs = make_instances(args.instances)
    log(f"generated {len(graphs)} instances, {sum(g.n for g in graphs)} nodes, {time.time() - t0:.1f} s")
    t1 = time.time()
    runs = fem_runs(graphs, R=args.replicas, T=args.label_steps, t_early=args.early_steps, stream=stream)
    torch.cuda.synchronize()
    log(f"ran plain FEM on the training set in {time.time() - t1:.1f} s")
    t2 = time.time()
    net, hist = train(graphs, runs, epochs=args.epochs)
    log(f"trained in {time.time() - t2:.1f} s")
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    net.save(args.out)
    print(json.dumps({"params": os.path.basename(args.out), "instances": len(graphs), "loss_per_epoch": hist,
                      "label_seconds": time.time() - t1, "train_seconds": time.time() - t2}))


if __name__ == "__main__":
    main()
