"""What the trained warm-start network gains over the method without it.

On held-out instances of the batched MaxCut recipe (seeds outside the
training and benchmark sets), the committed network
(paper_2412_09285_amd/data/mpnn_maxcut.bin) is compared with

* the plain anneal (R = 32, linear beta 0.01 -> 5 over 1000 steps), which
  defines the target: the sum over instances of its best cut, minus 0.1%;
* the same restart schedule without the network: after the first 100 plain
  steps the anneal continues (beta 0.3 -> 5 over 300 steps) from the fields
  themselves instead of the network's proposal.

Steps to target are counted with an anytime read-out every 25 steps.  The
GPU path is deterministic, so the outcome is fixed for the committed
parameters.
"""
import os

import numpy as np
import pytest

from paper_2412_09285_amd import fem
from paper_2412_09285_amd import workloads as W

pytestmark = pytest.mark.gpu

PARAMS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2412_09285_amd",
                      "data", "mpnn_maxcut.bin")
R, K, T_PLAIN, T_EARLY, T_WARM, BETA_START = 32, 25, 1000, 100, 300, 0.3


def anneal_to_target(solver, h, n_steps, target, best0=None):
    """Steps (multiple of K) until the sum of per-instance best cuts reaches
    target, or None; also the final per-instance best."""
    solver.set_fields(h)
    best = best0
    for b in range(K, n_steps + 1, K):
        solver.run_until(b)
        cur = solver.anytime_best().max(axis=1)
        best = cur if best is None else np.maximum(best, cur)
        if target is not None and best.sum() >= target:
            return b, best
    return None, best


@pytest.fixture(scope="module")
def setup():
    import torch

    sizes = np.exp(np.random.default_rng(3).uniform(np.log(1000), np.log(8000), size=24)).astype(int)
    graphs = [W.batch_instance(b, seed0=80_000, n_override=int(n)) for b, n in enumerate(sizes)]
    batch = fem.Problem.batch([fem.Problem.maxcut(g.n, g.u, g.v, g.w) for g in graphs])
    h0 = np.concatenate([W.initial_fields(g.n, R, seed=1_000_000 + g.meta["seed"]) for g in graphs])
    stream = torch.cuda.Stream()
    mk = lambda T, bmin=0.01: fem.Solver(batch, fem.default_params(replicas=R, steps=T, energy_every=0,
                                                                   eval_every=K, marginal_dtype=fem.BF16,
                                                                   beta_min=bmin), stream=stream)
    plain = mk(T_PLAIN)
    _, best_plain = anneal_to_target(plain, h0, T_PLAIN, None)
    target = float(np.sum(best_plain - 0.001 * np.abs(best_plain)))
    plain_steps, _ = anneal_to_target(plain, h0, T_PLAIN, target)
    # the state after the first T_EARLY plain steps, and the best seen so far
    plain.set_fields(h0)
    plain.run_until(T_EARLY)
    early_best = plain.anytime_best().max(axis=1)
    h_mid = plain.fields()
    return dict(batch=batch, mk=mk, target=target, plain_steps=plain_steps, h_mid=h_mid, early_best=early_best,
                best_plain=best_plain)


def test_network_reaches_target_sooner_than_plain_and_restart(setup):
    assert os.path.exists(PARAMS), "trained parameters missing"
    net = fem.MPNN(np.zeros(fem.N_MPNN_PARAMS, dtype=np.float32))
    net.load(PARAMS)
    prop = net.infer(setup["batch"], setup["h_mid"], seed=5, alpha=1.0)
    warm_steps, warm_best = anneal_to_target(setup["mk"](T_WARM, BETA_START), prop, T_WARM, setup["target"],
                                             setup["early_best"])
    restart_steps, restart_best = anneal_to_target(setup["mk"](T_WARM, BETA_START), setup["h_mid"], T_WARM,
                                                   setup["target"], setup["early_best"])
    tot = lambda s: None if s is None else T_EARLY + s
    print(f"[warm start] steps to target: plain {setup['plain_steps']}, network {tot(warm_steps)}, "
          f"restart without network {tot(restart_steps)}; best sums: network {warm_best.sum():.0f}, "
          f"restart {restart_best.sum():.0f}, target {setup['target']:.0f}", flush=True)
    # per instance: the relative gap of the best cut to plain FEM's at the
    # end of each continuation, and how many instances reach their own target
    bp = setup["best_plain"]
    gap = lambda best: (best - bp) / np.maximum(np.abs(bp), 1.0)
    at = lambda best: int(np.sum(best >= bp - 0.001 * np.abs(bp)))
    gw, gr = gap(warm_best), gap(restart_best)
    print(f"[warm start] per-instance gap to plain: network min {gw.min():.4f} median {np.median(gw):.4f} "
          f"max {gw.max():.4f}, {at(warm_best)}/{bp.size} at target; restart min {gr.min():.4f} "
          f"median {np.median(gr):.4f}, {at(restart_best)}/{bp.size} at target", flush=True)
    assert warm_steps is not None
    assert T_EARLY + warm_steps < setup["plain_steps"]
    assert restart_steps is None or restart_steps > warm_steps
    assert warm_best.sum() >= restart_best.sum()
    # the network helps the typical instance, not only the sum: its median
    # instance ends above plain FEM, and it leaves fewer instances below their
    # own target, by smaller gaps, than the restart without it (not every
    # instance reaches its target: see the two criteria of the benchmark)
    assert np.median(gw) > 0.0
    assert at(warm_best) >= at(restart_best)
    assert gw.min() >= gr.min()
