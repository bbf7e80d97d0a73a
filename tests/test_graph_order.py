"""The reverse Cuthill-McKee node order of fem_graph_order (host only): a
permutation of the nodes, the textbook bandwidths on paths and grids whatever
the input labels, components and isolated nodes handled, and a narrow band on
a 3-D random geometric graph in draw order."""
import numpy as np
import pytest

from paper_2412_09285_amd import fem
from paper_2412_09285_amd import workloads as W


def bandwidth(u, v):
    return int(np.max(np.abs(np.asarray(u, np.int64) - np.asarray(v, np.int64)))) if len(u) else 0


def shuffled(n, u, v, seed):
    perm = np.random.default_rng(seed).permutation(n).astype(np.int32)
    return perm[u], perm[v]


def test_path_gets_bandwidth_one():
    n = 500
    u, v = shuffled(n, np.arange(n - 1, dtype=np.int32), np.arange(1, n, dtype=np.int32), 1)
    assert bandwidth(u, v) > 10
    order = fem.graph_order(n, u, v)
    assert np.array_equal(np.sort(order), np.arange(n))
    assert bandwidth(*fem.relabel(order, u, v)) == 1


def test_grid_band_is_its_width():
    k = 30
    idx = np.arange(k * k).reshape(k, k)
    u = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()]).astype(np.int32)
    v = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()]).astype(np.int32)
    su, sv = shuffled(k * k, u, v, 2)
    order = fem.graph_order(k * k, su, sv)
    # breadth-first levels of a grid from a corner are its anti-diagonals, at
    # most k nodes each, and an edge spans at most two consecutive levels
    assert bandwidth(*fem.relabel(order, su, sv)) <= 2 * k


def test_components_isolated_nodes_and_determinism():
    # two paths and three isolated nodes
    u = np.array([0, 1, 2, 5, 6], np.int32)
    v = np.array([1, 2, 3, 6, 7], np.int32)
    n = 11
    o1 = fem.graph_order(n, u, v)
    o2 = fem.graph_order(n, u, v)
    assert np.array_equal(o1, o2)
    assert np.array_equal(np.sort(o1), np.arange(n))
    ru, rv = fem.relabel(o1, u, v)
    assert bandwidth(ru, rv) == 1


def test_rgg_band_narrows():
    g = W.rgg_3d(20000, 14.0, seed=5)
    before = np.abs(g.u.astype(np.int64) - g.v).mean()
    order = fem.graph_order(g.n, g.u, g.v)
    ru, rv = fem.relabel(order, g.u, g.v)
    after = np.abs(ru.astype(np.int64) - rv).mean()
    assert after < 0.1 * before, (before, after)


def test_invalid_edges_rejected():
    with pytest.raises(fem.FemError):
        fem.graph_order(3, np.array([0], np.int32), np.array([0], np.int32))
    with pytest.raises(fem.FemError):
        fem.graph_order(3, np.array([0], np.int32), np.array([5], np.int32))
