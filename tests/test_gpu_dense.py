"""GPU parity of the dense-W MaxCut path (matrix-core field product) against
the FP64 oracle, through the C ABI.

The oracle runs MaxCut on the same complete graph given as an edge list.  The
dense path forms phi = W m either exactly from int8 digit planes of the
fixed-point marginals (integral |W| <= 127, e.g. the +/-1 complete graphs
here) or with FP64 matrix-core products (any other W); both reproduce the
sparse kernel's FP64 accumulation, so the same 1e-5 lockstep tolerances
apply to gradients, energies and the propagated fields.  Also: ragged row and
replica blocks, the paper's K2000 optimiser setting (RMSprop with momentum,
inverse-proportional schedule), the full 2000-node size on sampled replicas,
the manipulated gradients (which run on the nonzero structure), captured
graphs, and argument checks.
"""
import numpy as np
import pytest

import oracle as O
from paper_2412_09285_amd import fem
from paper_2412_09285_amd import workloads as W
from _parity import grad_errors, lockstep

pytestmark = pytest.mark.gpu

K2000_OPT = dict(optimizer=fem.OPT_RMSPROP, momentum=0.63, rms_alpha=0.56, lr=0.03, weight_decay=0.013,
                 schedule=fem.SCHED_INVPROP, beta_min=1 / 1.16, beta_max=1 / 6e-5)


def oracle_params(R, T, kw):
    return O.Params(R=R, T=T, opt=kw.get("optimizer", 0), sched=kw.get("schedule", 0),
                    beta_min=kw.get("beta_min", 0.01), beta_max=kw.get("beta_max", 5.0), lr=kw.get("lr", 0.1),
                    wd=kw.get("weight_decay", 0.0), momentum=kw.get("momentum", 0.0),
                    rms_alpha=kw.get("rms_alpha", 0.99), manip=int(kw.get("gradient", 0) == fem.GRAD_MANIPULATED))


def lockstep_dense(g, R, T, n_steps, seed, tag, energies=True, **kw):
    h0 = W.initial_fields(g.n, R, seed)
    prob = fem.Problem.maxcut_dense(W.dense_matrix(g))
    s = fem.Solver(prob, fem.default_params(replicas=R, steps=T, keep_grad=1, **kw))
    P = oracle_params(R, T, kw)
    run = O.maxcut_run(g, P, h0)
    betas = [O.beta(P.sched, P.beta_min, P.beta_max, T, t) for t in range(n_steps)]
    return lockstep(s, run, P, n_steps, R, tag, betas, energies=energies)


def test_complete_pm1_first_100_steps():
    """K_300 with +/-1 weights (five row blocks, the last one partial), R = 70
    (two replica blocks, the second partial), Adam, linear schedule."""
    lockstep_dense(W.complete_pm1(300, seed=1), R=70, T=500, n_steps=100, seed=2, tag="dense K300")


def test_k2000_optimiser_setting():
    lockstep_dense(W.complete_pm1(256, seed=3), R=64, T=1000, n_steps=60, seed=4, tag="dense K256 rmsprop",
                   **K2000_OPT)


@pytest.mark.parametrize("n,R", [(1, 3), (2, 1), (64, 64), (65, 65), (130, 7)])
def test_edge_sizes(n, R):
    g = W.complete_pm1(n, seed=n) if n > 1 else W.Graph(1, np.zeros(0, np.int32), np.zeros(0, np.int32),
                                                        np.zeros(0, np.float32))
    lockstep_dense(g, R=R, T=100, n_steps=10, seed=n + R, tag=f"dense n{n} R{R}")


def test_fp64_path_complete_real_weights():
    """Non-integral weights take the FP64 matrix-core product: K_300, R = 70."""
    g = W.complete_pm1(300, seed=21)
    g.w = (g.w * np.random.default_rng(21).uniform(0.5, 1.5, size=g.n_edges)).astype(np.float32)
    lockstep_dense(g, R=70, T=500, n_steps=60, seed=22, tag="dense fp64 K300")


@pytest.mark.parametrize("wmax", [127, 128])
def test_integer_weight_range(wmax):
    """Integral weights up to 127 take the int8 digit path, 128 the FP64 one."""
    g = W.complete_pm1(200, seed=23)
    rng = np.random.default_rng(wmax)
    g.w = rng.integers(-wmax, wmax + 1, size=g.n_edges).astype(np.float32)
    g.w[0] = wmax
    lockstep_dense(g, R=40, T=300, n_steps=30, seed=24, tag=f"dense |W| <= {wmax}")


def test_weighted_near_complete():
    """Real weights and missing edges (a dense matrix with zeros)."""
    g = W.er_graph_m(200, 15000, seed=5, weights="one")
    g.w = np.random.default_rng(5).normal(size=g.n_edges).astype(np.float32)
    lockstep_dense(g, R=40, T=300, n_steps=30, seed=6, tag="dense weighted")


def test_manipulated_on_dense_problem():
    g = W.complete_pm1(150, seed=7)
    lockstep_dense(g, R=33, T=300, n_steps=30, seed=8, tag="dense manip", energies=False,
                   gradient=fem.GRAD_MANIPULATED, energy_every=0)


def test_full_size_sampled_replicas():
    """n = 2000, R = 1000 (the K2000 shape), two steps on the GPU; the
    replicas are independent, so the oracle runs a sample of them."""
    g = W.complete_pm1(2000, seed=9)
    R, T, steps = 1000, 1000, 2
    h0 = W.initial_fields(g.n, R, seed=10)
    prob = fem.Problem.maxcut_dense(W.dense_matrix(g))
    s = fem.Solver(prob, fem.default_params(replicas=R, steps=T, keep_grad=1, **K2000_OPT))
    s.set_fields(h0)
    s.step(steps)
    cols = np.array([0, 1, 63, 64, 500, 937, 998, 999])
    P = oracle_params(len(cols), T, K2000_OPT)
    run = O.maxcut_run(g, P, h0[:, cols])
    gh, _, _ = run.step(steps, record=True)
    rel, _ = grad_errors(s.last_grad()[:, cols], gh[-1], len(cols))
    hrel, _ = grad_errors(s.fields()[:, cols], run.h, len(cols))
    print(f"[dense K2000] sampled replicas: step-{steps - 1} grad rel err {rel.max():.2e}, h rel err {hrel.max():.2e}",
          flush=True)
    assert rel.max() <= 1e-5 and hrel.max() <= 1e-5


def test_capture_and_nt_flag_are_bitexact():
    g = W.complete_pm1(200, seed=11)
    R, T = 96, 40
    h0 = W.initial_fields(g.n, R, seed=12)
    prob = fem.Problem.maxcut_dense(W.dense_matrix(g))
    out = []
    for nt, graph in [(0, False), (1, False), (0, True), (1, True)]:
        s = fem.Solver(prob, fem.default_params(replicas=R, steps=T, energy_every=5, eval_every=5))
        vec, waves, rows, _, lanes = s.tile()
        s.set_tile(vec, waves, rows, nt, lanes)
        s.set_fields(h0)
        if graph:
            s.run_until(T)   # one captured graph
        else:
            s.step(T)        # eager launches
        out.append((s.fields(), s.anytime_best()))
    for f, b in out[1:]:
        assert np.array_equal(f, out[0][0]) and np.array_equal(b, out[0][1])


def test_dense_and_sparse_paths_agree():
    g = W.complete_pm1(256, seed=13)
    R, T = 64, 200
    h0 = W.initial_fields(g.n, R, seed=14)
    res = []
    for prob in (fem.Problem.maxcut(g.n, g.u, g.v, g.w), fem.Problem.maxcut_dense(W.dense_matrix(g))):
        s = fem.Solver(prob, fem.default_params(replicas=R, steps=T, eval_every=T))
        s.set_fields(h0)
        s.run_until(50)
        res.append(s.fields())
    rel, _ = grad_errors(res[1], res[0], R)
    assert rel.max() <= 1e-4, rel.max()


def test_argument_errors():
    Wm = W.dense_matrix(W.complete_pm1(10, seed=15))
    bad = Wm.copy(); bad[1, 2] = 3.0
    with pytest.raises(fem.FemError):
        fem.Problem.maxcut_dense(bad)
    bad = Wm.copy(); bad[4, 4] = 1.0
    with pytest.raises(fem.FemError):
        fem.Problem.maxcut_dense(bad)
    bad = Wm.copy(); bad[3, 5] = bad[5, 3] = np.nan
    with pytest.raises(fem.FemError):
        fem.Problem.maxcut_dense(bad)
    with pytest.raises(ValueError):
        fem.Problem.maxcut_dense(Wm[:, :9])
    prob = fem.Problem.maxcut_dense(Wm)
    with pytest.raises(fem.FemError):
        fem.Solver(prob, fem.default_params(replicas=4, steps=10, marginal_dtype=fem.BF16))
    with pytest.raises(fem.FemError):
        fem.Problem.batch([prob, prob])
