"""The seeded input generators (CPU): the structure each recipe promises
(edge counts, distinct pairs, no self-loops, weight sets, degree targets,
clause shapes, node-weight ranges), symmetry of the dense matrix, and that
every generator is a pure function of its seed."""
import numpy as np
import pytest

from paper_2412_09285_amd import workloads as W


def _pairs(g):
    assert np.all(g.u < g.v), "edges are listed with u < v"
    assert np.all((g.u >= 0) & (g.v < g.n))
    keys = g.u.astype(np.int64) * g.n + g.v
    return keys


def test_complete_pm1_and_dense_matrix():
    n = 57
    g = W.complete_pm1(n, seed=3)
    keys = _pairs(g)
    assert g.n_edges == n * (n - 1) // 2 and np.unique(keys).size == g.n_edges
    assert set(np.unique(g.w).tolist()) == {-1.0, 1.0}
    assert abs(float(np.mean(g.w))) < 0.1
    D = W.dense_matrix(g)
    assert D.dtype == np.float32 and D.shape == (n, n)
    assert np.array_equal(D, D.T) and np.all(np.diag(D) == 0)
    assert np.count_nonzero(D) == 2 * g.n_edges
    assert D[g.u[5], g.v[5]] == g.w[5]
    h = W.complete_pm1(n, seed=3)
    assert np.array_equal(h.w, g.w) and not np.array_equal(W.complete_pm1(n, seed=4).w, g.w)


def test_community_sizes():
    V = W.community_sizes(20000, seed=5, mean=4.0)
    assert V.dtype == np.int32 and V.min() >= 1
    assert abs(float(V.mean()) - 4.0) < 0.1
    assert np.array_equal(V, W.community_sizes(20000, seed=5, mean=4.0))


def test_sparse_graph_recipe():
    g = W.random_sparse_graph(5000, 15000, seed=7, weights="pm1")
    keys = _pairs(g)
    assert g.n_edges == 15000 and np.unique(keys).size == 15000
    assert set(np.unique(g.w).tolist()) <= {-1.0, 1.0}


def test_rgg_mean_degree():
    g = W.rgg_3d(20000, 14.0, seed=9)
    keys = _pairs(g)
    assert np.unique(keys).size == g.n_edges
    assert abs(2 * g.n_edges / g.n - 14.0) < 0.7
    assert np.all(g.w == 1.0)


def test_ksat_clauses():
    cnf = W.random_ksat(1000, 4000, 3, seed=2)
    assert cnf.n_clauses == 4000 and cnf.n_incidences == 12000
    lits = cnf.lits.reshape(-1, 3)
    var = np.abs(lits) - 1
    assert var.min() >= 0 and var.max() < 1000
    assert np.all((var[:, 0] != var[:, 1]) & (var[:, 0] != var[:, 2]) & (var[:, 1] != var[:, 2]))
    assert abs(float(np.mean(lits > 0)) - 0.5) < 0.03


@pytest.mark.parametrize("q", [1, 8])
def test_initial_fields(q):
    h = W.initial_fields(3000, 16, seed=1, q=q)
    assert h.dtype == np.float32 and h.shape == ((3000, 16) if q == 1 else (3000, 16, q))
    assert abs(float(np.std(h)) - 0.01) < 5e-4
    assert np.array_equal(h, W.initial_fields(3000, 16, seed=1, q=q))


def test_batch_instances_alternate_families():
    a = W.batch_instance(0, n_override=1000)
    b = W.batch_instance(1, n_override=1000)
    deg_a = np.bincount(np.concatenate([a.u, a.v]), minlength=a.n)
    assert np.all(deg_a == 3), "even instances are 3-regular"
    assert b.n_edges == 5 * b.n, "odd instances are G(n, 5n)"
    c = W.batch_instance(1, n_override=1000)
    assert np.array_equal(b.u, c.u) and np.array_equal(b.w, c.w)
