"""GPU parity of the node-weighted balance term (coarsened graphs whose nodes
carry community sizes V_i) against the FP64 oracle, through the C ABI:
lockstep fields, gradients and energies for the explicit and the manipulated
gradients, weighted group sizes, the best-replica criterion
2 cut + lambda (sum_s W_s^2 - sum_i V_i^2), batches mixing weighted and
unweighted parts, and argument checks."""
import numpy as np
import pytest

import oracle as O
from paper_2412_09285_amd import fem
from paper_2412_09285_amd import workloads as W
from _parity import lockstep

pytestmark = pytest.mark.gpu


def lockstep_weighted(g, V, q, R, T, n_steps, seed, lam, manip=False, tile=None, tag=""):
    h0 = W.initial_fields(g.n, R, seed, q=q)
    prob = fem.Problem.bmincut(g.n, g.u, g.v, g.w, q, node_weight=V)
    extra = dict(gradient=fem.GRAD_MANIPULATED, energy_every=0) if manip else {}
    s = fem.Solver(prob, fem.default_params(replicas=R, steps=T, keep_grad=1, lam=lam, **extra))
    if tile is not None:
        s.set_tile(*tile)
    P = O.Params(R=R, T=T, lam=lam, manip=int(manip))
    run = O.bmincut_run(g, q, P, h0, node_w=V)
    betas = [O.beta(0, P.beta_min, P.beta_max, T, t) for t in range(n_steps)]
    return lockstep(s, run, P, n_steps, R, tag, betas, energies=not manip)


@pytest.mark.parametrize("q", [4, 8])
def test_explicit_rgg_first_100_steps(q):
    g = W.rgg_3d(600, 14.0, seed=11)
    V = W.community_sizes(g.n, seed=12)
    lockstep_weighted(g, V, q, R=16, T=1000, n_steps=100, seed=13, lam=0.05, tag=f"weighted q{q}")


@pytest.mark.parametrize("q,R,n,tile", [(2, 3, 97, None), (16, 16, 333, (16, 2, 3, 0, 0)), (8, 64, 257, (8, 4, 2, 0, 4))])
def test_explicit_ragged(q, R, n, tile):
    g = W.random_sparse_graph(n, 3 * n, seed=q + n, weights="one")
    g.w = np.random.default_rng(q).integers(1, 4, size=g.n_edges).astype(np.float32)
    V = W.community_sizes(n, seed=n, mean=2.5)
    lockstep_weighted(g, V, q, R=R, T=300, n_steps=20, seed=q * 7 + R, lam=0.1, tile=tile, tag=f"n{n}_q{q}_R{R}")


@pytest.mark.parametrize("q", [4, 8])
def test_manipulated_rgg(q):
    g = W.rgg_3d(500, 14.0, seed=21)
    V = W.community_sizes(g.n, seed=22)
    lockstep_weighted(g, V, q, R=16, T=500, n_steps=60, seed=23, lam=0.05, manip=True, tag=f"manip weighted q{q}")


def test_sizes_and_best_criterion():
    rng = np.random.default_rng(4)
    g = W.rgg_3d(700, 12.0, seed=31)
    q, R, lam = 8, 12, 0.03
    V = W.community_sizes(g.n, seed=32)
    prob = fem.Problem.bmincut(g.n, g.u, g.v, g.w, q, node_weight=V)
    sigma = rng.integers(0, q, size=(R, g.n)).astype(np.int32)
    vals, sizes = prob.eval_int(sigma)
    assert np.array_equal(vals[0], O.cut(g.n, g.u, g.v, g.w, sigma).astype(np.int64))
    assert np.array_equal(sizes[0], O.group_sizes(g.n, q, sigma, node_w=V))
    h = W.initial_fields(g.n, R, seed=33, q=q) * 300.0
    s = fem.Solver(prob, fem.default_params(replicas=R, steps=5, lam=lam, eval_every=1))
    s.set_fields(h)
    sig = O.round_(h.astype(np.float64), q)
    cuts = O.cut(g.n, g.u, g.v, g.w, sig)
    Ws = O.group_sizes(g.n, q, sig, node_w=V).astype(np.float64)
    energy = 2 * cuts + lam * ((Ws ** 2).sum(1) - float(np.sum(V.astype(np.float64) ** 2)))
    rep, val, _ = s.best()
    assert rep[0] == int(np.argmin(energy)) and val[0] == int(cuts[rep[0]])
    s.step(1)   # anytime read-out of the fields after the step
    sig1 = O.round_(s.fields().astype(np.float64), q)
    Ws1 = O.group_sizes(g.n, q, sig1, node_w=V).astype(np.float64)
    e1 = 2 * O.cut(g.n, g.u, g.v, g.w, sig1) + lam * ((Ws1 ** 2).sum(1) - float(np.sum(V.astype(np.float64) ** 2)))
    assert np.array_equal(s.anytime_best()[0], e1)


def test_batch_mixes_weighted_and_unweighted_parts():
    q, R, lam, T = 4, 8, 0.1, 50
    gs = [W.rgg_3d(n, 10.0, seed=40 + n) for n in (200, 333, 150)]
    Vs = [W.community_sizes(gs[0].n, seed=41), None, W.community_sizes(gs[2].n, seed=43)]
    h0 = [W.initial_fields(g.n, R, seed=50 + b, q=q) for b, g in enumerate(gs)]
    parts = [fem.Problem.bmincut(g.n, g.u, g.v, g.w, q, node_weight=V) for g, V in zip(gs, Vs)]
    batch = fem.Problem.batch(parts)
    mk = lambda prob: fem.Solver(prob, fem.default_params(replicas=R, steps=T, lam=lam, eval_every=5))
    sb = mk(batch)
    sb.set_fields(np.concatenate(h0))
    sb.run_until(T)
    off = np.cumsum([0] + [g.n for g in gs])
    for b, (g, V) in enumerate(zip(gs, Vs)):
        s1 = mk(parts[b])
        s1.set_fields(h0[b])
        s1.run_until(T)
        assert np.array_equal(sb.fields()[off[b]:off[b + 1]], s1.fields()), b
        assert np.array_equal(sb.anytime_best()[b], s1.anytime_best()[0]), b


def test_unit_weights_match_unweighted_problem():
    g = W.rgg_3d(400, 12.0, seed=61)
    q, R = 8, 16
    h0 = W.initial_fields(g.n, R, seed=62, q=q)
    out = []
    for V in (None, np.ones(g.n, np.int32)):
        s = fem.Solver(fem.Problem.bmincut(g.n, g.u, g.v, g.w, q, node_weight=V),
                       fem.default_params(replicas=R, steps=30, lam=0.5, eval_every=3))
        s.set_fields(h0)
        s.run_until(30)
        out.append((s.fields(), s.anytime_best()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_argument_errors():
    g = W.rgg_3d(50, 6.0, seed=71)
    with pytest.raises(fem.FemError):
        fem.Problem.bmincut(g.n, g.u, g.v, g.w, 4, node_weight=np.zeros(g.n, np.int32))
    V = np.ones(g.n, np.int32)
    V[3] = -2
    with pytest.raises(fem.FemError):
        fem.Problem.bmincut(g.n, g.u, g.v, g.w, 4, node_weight=V)
    V = np.full(g.n, 1 << 20, np.int32)
    with pytest.raises(fem.FemError):
        fem.Problem.bmincut(g.n, g.u, g.v, g.w, 4, node_weight=V)
    with pytest.raises(ValueError):
        fem.Problem.bmincut(g.n, g.u, g.v, g.w, 4, node_weight=np.ones(g.n - 1, np.int32))
