"""GPU parity of the balanced min-cut (Potts, q states, softmax) hot path
against the FP64 oracle, through the C ABI.  Seeded inputs only; step parity
is lockstep along the oracle's trajectory (oracle -> GPU only)."""
import numpy as np
import pytest

import oracle as O
from paper_2412_09285_amd import fem
from paper_2412_09285_amd import workloads as W
from _parity import assert_energy_close, assert_grad_close, grad_errors, lockstep

pytestmark = pytest.mark.gpu


def free_run(g, q, R, T, n_steps, seed, lam=1.0, ramp=0, dtype=fem.F32, tile=None):
    h0 = W.initial_fields(g.n, R, seed, q=q)
    prob = fem.Problem.bmincut(g.n, g.u, g.v, g.w, q)
    s = fem.Solver(prob, fem.default_params(replicas=R, steps=T, keep_grad=1, record_energies=1, lam=lam,
                                            lambda_ramp=ramp, marginal_dtype=dtype))
    if tile is not None:
        s.set_tile(*tile)
    s.set_fields(h0)
    grads = []
    for _ in range(n_steps):
        s.step(1)
        grads.append(s.last_grad())
    U, S, F = s.energy_history(0, n_steps)
    run = O.bmincut_run(g, q, O.Params(R=R, T=T, lam=lam, lam_ramp=ramp), h0)
    gh, Uh, Sh = run.step(n_steps, record=True)
    betas = np.array([O.beta(0, 0.01, 5.0, T, t) for t in range(n_steps)])
    return dict(grads=np.array(grads), U=U[:, 0], S=S[:, 0], F=F[:, 0], h=s.fields(), gref=gh, Uref=Uh,
                Sref=Sh, href=run.h, betas=betas, h0=h0)


def lockstep_potts(g, q, R, T, n_steps, seed, lam=1.0, ramp=0, tile=None, tag="", dtype=fem.F32, sched=0,
                   beta_min=0.01, beta_max=5.0, tune=False):
    h0 = W.initial_fields(g.n, R, seed, q=q)
    prob = fem.Problem.bmincut(g.n, g.u, g.v, g.w, q)
    s = fem.Solver(prob, fem.default_params(replicas=R, steps=T, keep_grad=1, lam=lam, lambda_ramp=ramp,
                                            marginal_dtype=dtype, schedule=sched, beta_min=beta_min,
                                            beta_max=beta_max))
    if tile is not None:
        s.set_tile(*tile)
    if tune:
        s.set_fields(h0)
        tag += f", tile {s.tune(trial_steps=2, use_cache=True)}"
    P = O.Params(R=R, T=T, lam=lam, lam_ramp=ramp, mdt=int(dtype == fem.BF16), sched=sched, beta_min=beta_min,
                 beta_max=beta_max)
    run = O.bmincut_run(g, q, P, h0)
    betas = [O.beta(sched, P.beta_min, P.beta_max, T, t) for t in range(n_steps)]
    return lockstep(s, run, P, n_steps, R, tag, betas)


@pytest.mark.parametrize("q", [4, 8])
def test_rgg_q_first_100_steps(q):
    """3-D random geometric graph (mean degree 14, the bMinCut recipe at
    N = 600), lambda = 1 constant, R = 16: the first 100 steps."""
    lockstep_potts(W.rgg_3d(600, 14.0, seed=3), q, R=16, T=3000, n_steps=100, seed=103, tag=f"rgg600_q{q}")


@pytest.mark.parametrize("q,R,n", [(2, 3, 97), (16, 16, 333), (32, 5, 150), (8, 64, 257)])
def test_ragged(q, R, n):
    g = W.random_sparse_graph(n, 3 * n, seed=q + n, weights="one")
    g.w = np.random.default_rng(q).integers(1, 4, size=g.n_edges).astype(np.float32)
    lockstep_potts(g, q, R=R, T=300, n_steps=20, seed=q * 100 + R, lam=0.3, tag=f"n{n}_q{q}_R{R}")


def test_lambda_ramp():
    lockstep_potts(W.rgg_3d(300, 10.0, seed=5), 4, R=8, T=60, n_steps=60, seed=4, lam=0.8, ramp=1, tag="ramp")


@pytest.mark.parametrize("dtype", [fem.F32, fem.BF16])
def test_exponential_schedule_with_lambda_ramp(dtype):
    """The paper's bMinCut setting: exponential beta schedule and lambda
    ramped from 0 (Methods; supplementary bMinCut demonstration), q = 8:
    60 lockstep steps."""
    lockstep_potts(W.rgg_3d(500, 14.0, seed=12), 8, R=16, T=200, n_steps=60, seed=14, lam=0.5, ramp=1,
                   dtype=dtype, sched=fem.SCHED_EXP, beta_min=0.05, beta_max=30.0, tag=f"exp+ramp dtype {dtype}")


@pytest.mark.parametrize("q", [4, 8])
def test_rgg_bf16_first_100_steps(q):
    """BF16 copy of P: the first 100 steps against the oracle with the same
    bfloat16 copy, 1e-5 except where the two sides may round a marginal to
    different bfloat16 neighbours."""
    lockstep_potts(W.rgg_3d(600, 14.0, seed=3), q, R=16, T=3000, n_steps=100, seed=103, dtype=fem.BF16,
                   tag=f"rgg600_q{q} bf16")


@pytest.mark.parametrize("waves,rows,lanes", [(1, 1, 0), (8, 3, 0), (2, 16, 0), (4, 2, 4)])
def test_tile_shapes(waves, rows, lanes):
    lockstep_potts(W.rgg_3d(500, 14.0, seed=6), 8, R=16, T=100, n_steps=10, seed=8, tile=(8, waves, rows, 0, lanes),
                   tag=f"tile{waves}x{rows}L{lanes}")


@pytest.mark.parametrize("q,waves", [(2, 16), (4, 16), (16, 4)])
def test_largest_workgroups(q, waves):
    """The largest workgroup each q allows: the step kernel's per-lane LDS sums
    (q + 3 doubles per thread) are largest here (q = 4: 57 KB)."""
    lockstep_potts(W.rgg_3d(400, 12.0, seed=9), q, R=16, T=80, n_steps=8, seed=11, tile=(8, waves, 2, 0, 0),
                   tag=f"q{q}_waves{waves}")


def test_integer_eval_sizes_bitexact():
    rng = np.random.default_rng(1)
    g = W.rgg_3d(800, 12.0, seed=9)
    q = 8
    prob = fem.Problem.bmincut(g.n, g.u, g.v, g.w, q)
    sigma = rng.integers(0, q, size=(21, g.n)).astype(np.int32)
    vals, sizes = prob.eval_int(sigma)
    assert np.array_equal(vals[0], O.cut(g.n, g.u, g.v, g.w, sigma).astype(np.int64))
    assert np.array_equal(sizes[0], O.group_sizes(g.n, q, sigma))


def test_round_ties_lowest_state():
    g = W.rgg_3d(200, 8.0, seed=2)
    q, R = 4, 6
    h = W.initial_fields(g.n, R, seed=3, q=q)
    h[::5, :, 1] = h[::5, :, 2] = 5.0      # ties between states 1 and 2
    h[::7] = 0.0                           # all-equal rows -> state 0
    prob = fem.Problem.bmincut(g.n, g.u, g.v, g.w, q)
    s = fem.Solver(prob, fem.default_params(replicas=R, steps=5, lam=0.5))
    s.set_fields(h)
    assert np.array_equal(s.round(), O.round_(h.astype(np.float64), q))
    rep, val, _ = s.best()
    sig = O.round_(h.astype(np.float64), q)
    cuts = O.cut(g.n, g.u, g.v, g.w, sig)
    sz = O.group_sizes(g.n, q, sig)
    energy = 2 * cuts + 0.5 * (sz * (sz - 1)).sum(1)
    assert rep[0] == int(np.argmin(energy)) and val[0] == int(cuts[rep[0]])


def test_config3_full_size_two_steps():
    """N = 1,000,000 RGG (mean degree 14), q = 8, lambda = 1, R = 16 in the
    tuned launch shape: the first two steps lockstep with the oracle on all
    replicas at full size."""
    g = W.config_graph(3)
    q, R, T = 8, 16, 3000
    h0 = W.initial_fields(g.n, R, seed=103, q=q)
    prob = fem.Problem.bmincut(g.n, g.u, g.v, g.w, q)
    s = fem.Solver(prob, fem.default_params(replicas=R, steps=T, keep_grad=1, lam=1.0))
    s.set_fields(h0)
    tile = s.tune(trial_steps=2, use_cache=True)
    P = O.Params(R=R, T=T, lam=1.0)
    run = O.bmincut_run(g, q, P, h0)
    lockstep(s, run, P, 2, R, f"C3 full f32, tile {tile}", [O.beta(0, 0.01, 5.0, T, t) for t in range(2)])


def test_config3_full_size_bf16_two_steps():
    """The same at BF16 marginals (the recipe's storage type), all 16
    replicas: two lockstep steps against the oracle's bfloat16-copy mode."""
    lockstep_potts(W.config_graph(3), 8, R=16, T=3000, n_steps=2, seed=103, lam=1.0, dtype=fem.BF16,
                   tag="C3 full bf16", tune=True)
