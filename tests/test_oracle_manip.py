"""Pins of the oracle's manipulated gradients (supplementary "The explicit
gradient formulations" and "The explicit gradients and manipulated gradients
for the benchmarking problems").

The manipulated gradient is not the derivative of any free energy, so there
is no finite-difference check.  It is pinned instead by reductions to the
explicit gradient, which the finite-difference pins hold: where every
neighbour of a node is saturated (P_j exactly one-hot in double precision)
the one-hot vectors equal the marginals, and the manipulated gradient of that
node is the explicit one at a rescaled beta (and lambda), times a known
factor.  Further pins: the neighbours enter only through their read-out
(invariance under moves that keep it, the tie rule at h = 0), isolated nodes
keep only the entropy term, gamma scales linearly, and Max-k-SAT is left
unmodified.
"""
import numpy as np
import pytest

from paper_2412_09285_amd import workloads as W


def bipartite_biregular(nA, nB, d, seed):
    """Every B node joined to d distinct A nodes, +/-1 weights; each edge is
    listed with a random orientation."""
    rng = np.random.default_rng(seed)
    u, v = [], []
    for b in range(nB):
        for a in rng.choice(nA, size=d, replace=False):
            x, y = (int(a), nA + b) if rng.random() < 0.5 else (nA + b, int(a))
            u.append(x)
            v.append(y)
    w = rng.choice([-1.0, 1.0], size=len(u))
    return W.Graph(nA + nB, np.array(u, np.int32), np.array(v, np.int32), w.astype(np.float32))


@pytest.mark.parametrize("gamma", [1.0, 0.37])
def test_maxcut_manip_reduces_to_explicit_at_saturated_neighbours(orc, gamma):
    nA, nB, d, R = 30, 25, 4, 5
    g = bipartite_biregular(nA, nB, d, seed=3)
    rng = np.random.default_rng(4)
    h = np.empty((g.n, R))
    h[:nA] = rng.choice([-60.0, 60.0], size=(nA, R))     # tanh(30) == 1 in double
    h[nA:] = rng.normal(0.0, 1.5, size=(nB, R))
    beta = 0.8
    gm = orc.maxcut_grad_manip(g.n, g.u, g.v, g.w, h, beta, gamma)
    # c_i = 1/d on B; manipulated = gamma (c/2) explicit(beta' = beta c / 2)
    c = 1.0 / d
    gp, _, _ = orc.maxcut_grad(g.n, g.u, g.v, g.w, h, beta * c / 2.0)
    ref = gamma * (c / 2.0) * gp[nA:]
    np.testing.assert_allclose(gm[nA:], ref, rtol=1e-12, atol=1e-15 * np.abs(ref).max())
    assert np.abs(ref).max() > 1e-3


def test_bmincut_manip_reduces_to_explicit_at_saturated_neighbours(orc):
    q, R, lam, beta, gamma = 4, 3, 0.7, 1.3, 0.9
    g = W.rgg_3d(40, 6.0, seed=11)
    rng = np.random.default_rng(12)
    w = rng.uniform(0.5, 2.0, size=g.u.shape[0])
    D = np.zeros(g.n)
    np.add.at(D, g.u, w)
    np.add.at(D, g.v, w)
    tested = 0
    for i in np.argsort(-D)[:6]:
        if D[i] == 0:
            continue
        # every node but i exactly one-hot (exp(-1000) == 0), node i generic
        h = np.full((g.n, R, q), -1000.0)
        states = rng.integers(0, q, size=(g.n, R))
        for j in range(g.n):
            h[j, np.arange(R), states[j]] = 0.0
        h[i] = rng.normal(0.0, 1.0, size=(R, q))
        gm = orc.bmincut_grad_manip(g.n, g.u, g.v, w, q, lam, h, beta, gamma)
        # ghat = k g^p with k = c^f/2, lambda' = lambda c^a/c^f = lambda sqrt(D), beta' = k beta
        k = (q / D[i]) / 2.0
        gp, _, _ = orc.bmincut_grad(g.n, g.u, g.v, w, q, lam * np.sqrt(D[i]), h, k * beta)
        ref = gamma * k * gp[i]
        np.testing.assert_allclose(gm[i], ref, rtol=1e-10, atol=1e-13 * np.abs(ref).max())
        tested += 1
    assert tested >= 4


def test_maxcut_manip_sees_only_the_readout(orc):
    g0_ = W.random_sparse_graph(60, 200, seed=5, weights="pm1")
    rng = np.random.default_rng(6)
    g = W.Graph(g0_.n, g0_.u, g0_.v, rng.normal(0.0, 1.0, size=g0_.u.shape[0]).astype(np.float32))
    h = rng.normal(0.0, 1.0, size=(g.n, 4))
    beta = 0.6
    g0 = orc.maxcut_grad_manip(g.n, g.u, g.v, g.w, h, beta)
    # rescale every field but keep its sign: only own terms change
    h2 = h * rng.uniform(0.1, 3.0, size=h.shape)
    g2 = orc.maxcut_grad_manip(g.n, g.u, g.v, g.w, h2, beta)
    P = 1.0 / (1.0 + np.exp(-h))
    P2 = 1.0 / (1.0 + np.exp(-h2))
    field = g0 / (P * (1 - P)) - h / beta      # c_i sum_j W_ij sgn(m_j)
    field2 = g2 / (P2 * (1 - P2)) - h2 / beta
    np.testing.assert_allclose(field, field2, rtol=1e-9, atol=1e-12)
    # tie rule: h_j = 0 reads out as (-), like h_j < 0 (both edge orientations)
    for j, nb in ((int(g.u[0]), int(g.v[0])), (int(g.v[1]), int(g.u[1]))):
        hz, hn, hp = h.copy(), h.copy(), h.copy()
        hz[j, 0], hn[j, 0], hp[j, 0] = 0.0, -0.25, 0.25
        gz = orc.maxcut_grad_manip(g.n, g.u, g.v, g.w, hz, beta)
        gn = orc.maxcut_grad_manip(g.n, g.u, g.v, g.w, hn, beta)
        gpos = orc.maxcut_grad_manip(g.n, g.u, g.v, g.w, hp, beta)
        assert gz[nb, 0] == gn[nb, 0]
        assert gz[nb, 0] != gpos[nb, 0]


def test_bmincut_manip_ties_go_to_the_lowest_state(orc):
    g = W.Graph(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([1.0, 2.0], np.float32))
    q = 3
    h = np.zeros((3, 1, q))
    h[0, 0] = [0.2, -0.1, 0.4]
    h[2, 0] = [-0.3, 0.5, 0.1]
    # node 1 tied between states 1 and 2 -> read-out state 1; same as a clear win of state 1
    h_tie = h.copy()
    h_tie[1, 0] = [-1.0, 0.5, 0.5]
    h_win = h.copy()
    h_win[1, 0] = [-1.0, 0.9, 0.5]
    a = orc.bmincut_grad_manip(3, g.u, g.v, g.w, q, 0.5, h_tie, 1.0)
    b = orc.bmincut_grad_manip(3, g.u, g.v, g.w, q, 0.5, h_win, 1.0)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[2], b[2])


def test_isolated_nodes_keep_only_entropy(orc):
    g = W.Graph(5, np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([1.0, -1.0], np.float32))
    h = np.array([[0.3, -1.2], [0.1, 0.0], [-0.4, 2.0], [0.7, -0.9], [-1.1, 0.05]])
    beta, gamma = 2.0, 1.7
    gm = orc.maxcut_grad_manip(5, g.u, g.v, g.w, h, beta, gamma)
    P = 1.0 / (1.0 + np.exp(-h[3:]))
    np.testing.assert_allclose(gm[3:], gamma * P * (1 - P) * h[3:] / beta, rtol=1e-13)
    gq = W.Graph(4, np.array([0], np.int32), np.array([1], np.int32), np.array([1.0], np.float32))
    hq = np.random.default_rng(1).normal(size=(4, 2, 3))
    gb = orc.bmincut_grad_manip(4, gq.u, gq.v, gq.w, 3, 0.8, hq, beta, gamma)
    for i in (2, 3):   # isolated: c^f = c^a = 0, only (ln P + 1)/beta remains
        Pq = np.exp(hq[i]) / np.exp(hq[i]).sum(axis=1, keepdims=True)
        A = np.log(Pq) / beta
        np.testing.assert_allclose(gb[i], gamma * Pq * (A - (Pq * A).sum(axis=1, keepdims=True)), rtol=1e-12,
                                   atol=1e-15)


def test_gamma_is_linear_and_sat_is_unmodified(orc):
    g = W.random_sparse_graph(50, 150, seed=8, weights="pm1")
    h = np.random.default_rng(9).normal(size=(g.n, 3))
    a = orc.maxcut_grad_manip(g.n, g.u, g.v, g.w, h, 1.1, 1.0)
    b = orc.maxcut_grad_manip(g.n, g.u, g.v, g.w, h, 1.1, 2.5)
    np.testing.assert_allclose(b, 2.5 * a, rtol=1e-14)
    cnf = W.random_ksat(40, 160, 3, seed=10)
    hs = np.random.default_rng(11).normal(size=(40, 3))
    gs, _, _ = orc.maxsat_grad(40, cnf.clause_off, cnf.lits, hs, 0.9)
    gm = orc.maxsat_grad_manip(40, cnf.clause_off, cnf.lits, hs, 0.9, 0.6)
    np.testing.assert_allclose(gm, 0.6 * gs, rtol=1e-14)


def test_manip_run_follows_eval_and_optimiser(orc):
    """The annealing loop in manipulated mode applies Adam to the manipulated
    gradient of each step."""
    g = W.random_sparse_graph(80, 240, seed=12, weights="pm1")
    R, T = 4, 30
    h0 = W.initial_fields(g.n, R, seed=13)
    P = orc.Params(R=R, T=T, manip=1, gamma=0.8)
    run = orc.maxcut_run(g, P, h0)
    h, m1, m2 = run.h.copy(), run.m1.copy(), run.m2.copy()
    for t in range(5):
        gg, U, S = run.eval_at(h, t)
        assert U is None and S is None
        orc.adam(gg, h, m1, m2, P.lr, P.b1, P.b2, P.eps, P.wd, t + 1)
    run.step(5)
    np.testing.assert_array_equal(run.h, h)
