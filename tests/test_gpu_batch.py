"""GPU parity of the batched launch against one FP64 oracle run per instance.

Replicas of different instances are independent mean-field solutions, so a
block-diagonal batch of instances stepped together must give, instance by
instance, what the oracle gives for that instance alone (Results,
"Free-Energy Machine": replicas updated in parallel).  The batch is stepped
lockstep from the oracle's per-instance states (oracle -> GPU only); each
instance's gradient, energies, h(t+1) and anytime best are judged against its
own oracle run, for MaxCut, bMinCut and Max-k-SAT with float32 and bfloat16
marginal copies.  At the full 512-instance workload (R = 32, bfloat16, the
launch shape the benchmark times) the first step is checked on sampled
instances, with the read-out of every instance's best replica.
"""
import numpy as np
import pytest

import oracle as O
from paper_2412_09285_amd import fem
from paper_2412_09285_amd import workloads as W
from _parity import assert_energy_close, assert_grad_close, bf16_slack, lockstep_batch, u_scale

pytestmark = pytest.mark.gpu


def _check_anytime(s, ref_best, undecided, tag):
    got = s.anytime_best()
    ok = ~undecided
    assert np.array_equal(got[ok], ref_best[ok]), f"{tag}: anytime best differs from the oracle's read-outs"


def _check_best(s, runs, offsets, h_parts, q=1):
    """fem_best on the oracle's own fields: per instance the best replica and
    its value, bit-exact (both sides round the same float32 fields)."""
    s.set_fields(np.concatenate(h_parts).astype(np.float32))
    rep, val, sig = s.best()
    for b, (run, h) in enumerate(zip(runs, h_parts)):
        sigma = O.round_(h.astype(np.float32).astype(np.float64), q)
        from _parity import instance_value
        v = instance_value(run, sigma)
        if run.kind == O.KIND_MAXCUT:
            r = int(np.argmax(v))
        else:
            r = int(np.argmin(v))
        assert rep[b] == r, (b, rep[b], r)
        if run.kind == O.KIND_BMINCUT:
            u, vv, w = run._keep
            assert val[b] == int(O.cut(run.n, u, vv, w, sigma[r:r + 1])[0])
        else:
            assert val[b] == int(v[r])
        assert np.array_equal(sig[offsets[b]:offsets[b + 1]], sigma[r])


def _graphs_c5_like(sizes, seed0):
    return [W.batch_instance(b, seed0=seed0, n_override=int(n)) for b, n in enumerate(sizes)]


@pytest.mark.parametrize("dtype", [fem.F32, fem.BF16])
def test_maxcut_batch_equals_oracle_per_instance(dtype):
    """Five uneven instances of the batched MaxCut recipe (3-regular and
    G(n, 5n), +/-1 weights; 60..1000 nodes), R = 32: 30 batched lockstep
    steps against five oracle runs."""
    graphs = _graphs_c5_like([60, 333, 1000, 97, 512], seed0=91_000)
    R, T, n_steps = 32, 1000, 30
    batch = fem.Problem.batch([fem.Problem.maxcut(g.n, g.u, g.v, g.w) for g in graphs])
    offsets = batch.instance_offsets()
    s = fem.Solver(batch, fem.default_params(replicas=R, steps=T, keep_grad=1, eval_every=1, marginal_dtype=dtype))
    P = O.Params(R=R, T=T, mdt=int(dtype == fem.BF16))
    runs = [O.maxcut_run(g, P, W.initial_fields(g.n, R, seed=1_000_000 + g.meta["seed"])) for g in graphs]
    betas = [O.beta(0, P.beta_min, P.beta_max, T, t) for t in range(n_steps)]
    _, ref_best, und = lockstep_batch(s, runs, offsets, P, n_steps, R, f"maxcut batch dtype {dtype}", betas)
    _check_anytime(s, ref_best, und, "maxcut batch")
    _check_best(s, runs, offsets, [r.h for r in runs])


@pytest.mark.parametrize("dtype", [fem.F32, fem.BF16])
def test_bmincut_batch_equals_oracle_per_instance(dtype):
    """Four uneven 3-D RGG instances (70..400 nodes), q = 4, lambda = 0.3,
    R = 8: 20 batched lockstep steps against four oracle runs."""
    graphs = [W.rgg_3d(n, 10.0, seed=40 + n) for n in (70, 400, 151, 260)]
    q, R, T, n_steps = 4, 8, 200, 20
    batch = fem.Problem.batch([fem.Problem.bmincut(g.n, g.u, g.v, g.w, q) for g in graphs])
    offsets = batch.instance_offsets()
    s = fem.Solver(batch, fem.default_params(replicas=R, steps=T, keep_grad=1, eval_every=1, lam=0.3,
                                            marginal_dtype=dtype))
    P = O.Params(R=R, T=T, lam=0.3, mdt=int(dtype == fem.BF16))
    runs = [O.bmincut_run(g, q, P, W.initial_fields(g.n, R, seed=g.n, q=q)) for g in graphs]
    betas = [O.beta(0, P.beta_min, P.beta_max, T, t) for t in range(n_steps)]
    _, ref_best, und = lockstep_batch(s, runs, offsets, P, n_steps, R, f"bmincut batch dtype {dtype}", betas)
    _check_anytime(s, ref_best, und, "bmincut batch")
    _check_best(s, runs, offsets, [r.h for r in runs], q=q)


@pytest.mark.parametrize("dtype", [fem.F32, fem.BF16])
def test_maxsat_batch_equals_oracle_per_instance(dtype):
    """Four uneven random 3-SAT instances (50..800 variables, ratio 6),
    R = 16: 20 batched lockstep steps against four oracle runs."""
    cnfs = [W.random_ksat(n, 6 * n, 3, seed=n) for n in (50, 800, 123, 400)]
    R, T, n_steps = 16, 300, 20
    batch = fem.Problem.batch([fem.Problem.maxsat(c.n_vars, c.clause_off, c.lits) for c in cnfs])
    offsets = batch.instance_offsets()
    s = fem.Solver(batch, fem.default_params(replicas=R, steps=T, keep_grad=1, eval_every=1, marginal_dtype=dtype))
    P = O.Params(R=R, T=T, mdt=int(dtype == fem.BF16))
    runs = [O.maxsat_run(c, P, W.initial_fields(c.n_vars, R, seed=c.n_vars + 1)) for c in cnfs]
    betas = [O.beta(0, P.beta_min, P.beta_max, T, t) for t in range(n_steps)]
    _, ref_best, und = lockstep_batch(s, runs, offsets, P, n_steps, R, f"maxsat batch dtype {dtype}", betas)
    _check_anytime(s, ref_best, und, "maxsat batch")
    _check_best(s, runs, offsets, [r.h for r in runs])


def test_full_512_instance_batch_first_step_sampled():
    """The benchmark's batch: 512 MaxCut instances (N log-uniform in
    [1000, 50000]), R = 32, bfloat16 copy, energies on, in the launch shape
    the benchmark uses.  Step 0 from h0 on the whole batch; on eight sampled
    instances (the smallest, the largest and six seeded picks) the gradient
    and energies against the oracle, and on every instance the read-out of
    the best replica of h0 against the oracle."""
    from paper_2412_09285_amd import batchbench as BB

    graphs = BB.instances(512)
    R, T = 32, 1000
    parts = [fem.Problem.maxcut(g.n, g.u, g.v, g.w) for g in graphs]
    batch = fem.Problem.batch(parts)
    offsets = batch.instance_offsets()
    h0s = [BB.h0_for(g, R) for g in graphs]
    h0 = np.concatenate(h0s)
    s = fem.Solver(batch, fem.default_params(replicas=R, steps=T, keep_grad=1, energy_every=1,
                                            marginal_dtype=fem.BF16))
    s.set_fields(h0)
    tile = s.tune(trial_steps=5, use_cache=True)
    s.set_fields(h0)
    s.step(1)
    g = s.last_grad().astype(np.float64)
    U, S, F = s.energies()
    sizes = np.array([gr.n for gr in graphs])
    picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)),
                    *np.random.default_rng(17).choice(512, size=6, replace=False).tolist()})
    P = O.Params(R=R, T=T, mdt=1)
    for b in picks:
        run = O.maxcut_run(graphs[b], P, h0s[b])
        h = h0s[b].astype(np.float64)
        gref, Uref, Sref = run.eval_at(h, 0)
        gslack, uslack = bf16_slack(run, h, 0)
        assert_grad_close(g[offsets[b]:offsets[b + 1]], gref, R, what=f"C5 instance {b} g", slack=gslack)
        assert_energy_close(U[b], S[b], F[b], Uref, Sref, O.beta(0, 0.01, 5.0, T, 0), what=f"C5 instance {b}",
                            uscale=u_scale(run, h, 0), uslack=uslack)
    # read-out of h0: the best replica of every instance, bit-exact
    s.set_fields(h0)
    rep, val, _ = s.best()
    for b in range(512):
        gr = graphs[b]
        cuts = O.cut(gr.n, gr.u, gr.v, gr.w, O.round_(h0s[b].astype(np.float64), 1))
        assert rep[b] == int(np.argmax(cuts)) and val[b] == int(cuts.max()), b
    print(f"[C5 full batch] step 0 on instances {picks} within the bar; best replica of h0 exact on all 512; "
          f"tile {tile}", flush=True)
