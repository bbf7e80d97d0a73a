"""Pins of the node-weighted balance term (supplementary chip-partitioning
section: coarsened nodes carry node weights V_i, and the balance term sums
V_i V_j P_i P_j over i != j): unit weights reproduce the unweighted oracle
bit for bit; the energy equals the expectation of the weighted energy over
all configurations; the gradient matches finite differences of F; the
manipulated form reduces to the explicit one at saturated neighbours; group
sizes sum the weights."""
import itertools
import math

import numpy as np
import pytest

from paper_2412_09285_amd import workloads as W
from test_oracle_pins import _fd_check, small_graph


def weighted_E(sig, u, v, w, V, lam, q):
    """2 cut + lam (sum_s W_s^2 - sum_i V_i^2), W_s = total weight in state s:
    the ordered-pair cut plus lam sum_{i != j, same state} V_i V_j."""
    cut = 2.0 * sum(wi for a, b, wi in zip(u, v, w) if sig[a] != sig[b])
    Ws = np.zeros(q)
    for i, s in enumerate(sig):
        Ws[s] += V[i]
    return cut + lam * (float(np.sum(Ws ** 2)) - float(np.sum(np.asarray(V, float) ** 2)))


def test_unit_weights_reproduce_unweighted(orc):
    g = small_graph(10, 20, seed=2)
    g.w = np.random.default_rng(2).uniform(0.2, 2, size=g.n_edges)
    h = np.random.default_rng(3).normal(size=(10, 3, 4))
    a = orc.bmincut_grad(10, g.u, g.v, g.w, 4, 0.6, h, 0.9)
    b = orc.bmincut_grad(10, g.u, g.v, g.w, 4, 0.6, h, 0.9, node_w=np.ones(10))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert np.array_equal(orc.bmincut_grad_manip(10, g.u, g.v, g.w, 4, 0.6, h, 0.9),
                          orc.bmincut_grad_manip(10, g.u, g.v, g.w, 4, 0.6, h, 0.9, node_w=np.ones(10)))


@pytest.mark.parametrize("q,n,lam", [(3, 5, 0.7), (2, 6, 0.4)])
def test_weighted_energy_vs_enumeration(orc, q, n, lam):
    g = small_graph(n, 7, seed=q * 10 + n)
    g.w = np.random.default_rng(q).uniform(0.2, 2, size=g.n_edges)
    V = np.random.default_rng(q + 1).integers(1, 5, size=n).astype(float)
    R = 2
    h = np.random.default_rng(7).normal(0, 1.2, size=(n, R, q))
    _, U, S = orc.bmincut_grad(n, g.u, g.v, g.w, q, lam, h, 1.1, node_w=V)
    for r in range(R):
        P = np.exp(h[:, r, :]) / np.exp(h[:, r, :]).sum(1, keepdims=True)
        EU, ES = 0.0, 0.0
        for sig in itertools.product(range(q), repeat=n):
            pr = float(np.prod([P[i, s] for i, s in enumerate(sig)]))
            EU += pr * weighted_E(sig, g.u, g.v, g.w, V, lam, q)
            ES -= pr * math.log(pr)
        assert abs(U[r] - EU) <= 1e-11 * max(1.0, abs(EU))
        assert abs(S[r] - ES) <= 1e-11 * max(1.0, abs(ES))


def test_weighted_gradient_fd(orc):
    n, q, lam = 9, 4, 0.3
    g = small_graph(n, 20, seed=5)
    g.w = np.random.default_rng(5).uniform(0.2, 2, size=g.n_edges)
    V = np.random.default_rng(6).integers(1, 6, size=n).astype(float)
    h = np.random.default_rng(9).normal(0, 1.0, size=(n, 2, q))
    _fd_check(lambda hh, b: orc.bmincut_grad(n, g.u, g.v, g.w, q, lam, hh, b, node_w=V), h, 1.3)


def test_weighted_manip_reduces_to_explicit(orc):
    q, R, lam, beta, gamma = 4, 3, 0.7, 1.3, 0.9
    g = W.rgg_3d(40, 6.0, seed=11)
    rng = np.random.default_rng(12)
    w = rng.uniform(0.5, 2.0, size=g.u.shape[0])
    V = rng.integers(1, 7, size=g.n).astype(float)
    D = np.zeros(g.n)
    np.add.at(D, g.u, w)
    np.add.at(D, g.v, w)
    for i in np.argsort(-D)[:4]:
        h = np.full((g.n, R, q), -1000.0)
        states = rng.integers(0, q, size=(g.n, R))
        for j in range(g.n):
            h[j, np.arange(R), states[j]] = 0.0
        h[i] = rng.normal(0.0, 1.0, size=(R, q))
        gm = orc.bmincut_grad_manip(g.n, g.u, g.v, w, q, lam, h, beta, gamma, node_w=V)
        k = (q / D[i]) / 2.0
        gp, _, _ = orc.bmincut_grad(g.n, g.u, g.v, w, q, lam * np.sqrt(D[i]), h, k * beta, node_w=V)
        np.testing.assert_allclose(gm[i], gamma * k * gp[i], rtol=1e-10, atol=1e-13 * np.abs(gp[i]).max())


def test_weighted_group_sizes(orc):
    rng = np.random.default_rng(1)
    n, q, R = 30, 5, 4
    V = rng.integers(1, 9, size=n).astype(np.int32)
    sig = rng.integers(0, q, size=(R, n)).astype(np.int32)
    sizes = orc.group_sizes(n, q, sig, node_w=V)
    for r in range(R):
        for s in range(q):
            assert sizes[r, s] == int(V[sig[r] == s].sum())
    assert np.array_equal(orc.group_sizes(n, q, sig), orc.group_sizes(n, q, sig, node_w=np.ones(n, np.int32)))
