"""Pins of the FP64 reference of the warm-start network: the Philox generator
against its published known-answer vectors, bfloat16 rounding against its
definition, the state features at closed-form points, the analytic backward
pass against central finite differences of the loss, and the independence of
the instances of a block-diagonal batch."""
import json
import os

import numpy as np
import pytest

from oracle import mpnn as M
from paper_2412_09285_amd import workloads as W


def test_philox_known_answers():
    kat = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "philox_kat.json")))
    for v in kat["vectors"]:
        c = [int(x, 16) for x in v["counter"]]
        k = [int(x, 16) for x in v["key"]]
        out = M.philox4x32_10(*[np.uint64(x) for x in c], k[0], k[1])
        assert [int(x) for x in out] == [int(x, 16) for x in v["out"]]


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3e-39], dtype=np.float32)
    r = M.bf16_round(x)
    # ties to even: 1 + 2^-8 -> 1 ; 1 + 2^-7 + 2^-8 -> 1 + 2^-6 ; 1 + 3*2^-9 -> 1 + 2^-7
    assert list(r[:5]) == [1.0, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7, -2.5]
    # bf16 keeps 8 significant bits: relative error <= 2^-8
    y = np.random.default_rng(0).normal(size=1000).astype(np.float32)
    assert np.all(np.abs(M.bf16_round(y) - y) <= 2.0 ** -8 * np.abs(y) + 1e-40)


def test_features_closed_forms_and_random_columns():
    ops = M.GraphOps(50, np.array([0, 1]), np.array([1, 2]), np.array([1.0, -1.0]))
    state = np.zeros(50, dtype=np.float32)
    state[:5] = [0.0, 2.0 * np.log(3.0), -10.0, 10.0, -1.0]
    x = M.features(ops, state, seed=123, draw=4)
    assert np.all(x[:, 0] == 1.0)
    assert x[0, 1] == pytest.approx(np.log(2.0)) and x[1, 1] == pytest.approx(np.log(3.0)) and x[3, 1] == 0.0
    assert x[0, 2] == 1.0 and x[1, 2] == 0.0 and x[3, 2] == 0.0
    # tanh(ln 3) = (9 - 1) / (9 + 1)
    assert x[0, 3] == 0.0 and x[1, 3] == pytest.approx(0.8, rel=1e-6) and x[2, 3] == pytest.approx(-1.0, abs=1e-4)
    assert list(x[:5, 4]) == pytest.approx([0.0, np.log(3.0) / 2.0, -2.0, 2.0, -0.25], rel=1e-6)
    assert np.all((x[:, 5:] >= -1) & (x[:, 5:] < 1))
    assert np.array_equal(x[:, 5:].astype(np.float32).astype(np.float64), x[:, 5:])
    # the uniforms depend on the draw and the seed, not on the state
    y = M.features(ops, state * 3, seed=123, draw=4)
    assert np.array_equal(x[:, 5:], y[:, 5:])
    assert not np.array_equal(x[:, 5:], M.features(ops, state, seed=123, draw=5)[:, 5:])
    assert not np.array_equal(x[:, 5:], M.features(ops, state, seed=124, draw=4)[:, 5:])


def union(gs):
    off = np.cumsum([0] + [g.n for g in gs])
    u = np.concatenate([g.u + off[b] for b, g in enumerate(gs)])
    v = np.concatenate([g.v + off[b] for b, g in enumerate(gs)])
    w = np.concatenate([g.w for g in gs])
    return M.GraphOps(int(off[-1]), u, v, w), off


@pytest.fixture(scope="module")
def small_batch():
    gs = [W.random_sparse_graph(40 + 7 * b, 90 + 10 * b, seed=b, weights="pm1") for b in range(3)]
    ops, off = union(gs)
    rng = np.random.default_rng(4)
    state = rng.normal(0.0, 2.0, size=ops.n).astype(np.float32)
    y = rng.integers(0, 2, size=ops.n).astype(np.float64)
    return ops, off, state, y


def test_backward_matches_finite_differences(small_batch):
    ops, off, state, y = small_batch
    theta = W.mpnn_init_weights(7).astype(np.float64)
    L, grad, Ls = M.batch_loss_and_grad(ops, off, state, y, theta, 99, 3, quantize=False)
    assert L == pytest.approx(M.batch_loss(ops, off, state, y, theta, 99, 3, quantize=False), rel=1e-14)
    rng = np.random.default_rng(1)
    eps = 1e-6
    idx = []
    k = 0
    for name, shp in M.SHAPES:   # every parameter block, a few coordinates each
        n = int(np.prod(shp))
        idx += list(k + rng.choice(n, size=min(n, 6), replace=False))
        k += n
    f = lambda th: M.batch_loss(ops, off, state, y, th, 99, 3, quantize=False)
    for j in idx:
        tp = theta.copy(); tp[j] += eps
        tm = theta.copy(); tm[j] -= eps
        fd = (f(tp) - f(tm)) / (2 * eps)
        assert abs(fd - grad[j]) <= 1e-6 * max(1.0, abs(grad).max()), (j, fd, grad[j])
    # directional derivative along a unit direction, with a step small enough
    # that no pre-activation crosses zero (the ReLU kinks)
    dv = rng.normal(size=theta.size)
    dv /= np.linalg.norm(dv)
    e2 = 1e-7
    fd = (f(theta + e2 * dv) - f(theta - e2 * dv)) / (2 * e2)
    assert fd == pytest.approx(float(grad @ dv), rel=1e-5, abs=1e-10)


def test_batch_instances_are_independent(small_batch):
    """Messages never cross instances: changing one instance's state or
    labels leaves the other instances' logits and losses unchanged, and the
    batch gradient is the mean of the per-instance gradients."""
    ops, off, state, y = small_batch
    theta = W.mpnn_init_weights(11).astype(np.float64)
    z = M.forward(ops, theta, state, 7, 2)["z"]
    s2 = state.copy()
    s2[off[0]:off[1]] *= -3.0
    z2 = M.forward(ops, theta, s2, 7, 2)["z"]
    assert np.array_equal(z[off[1]:], z2[off[1]:])
    assert not np.array_equal(z[:off[1]], z2[:off[1]])
    L, g, Ls = M.batch_loss_and_grad(ops, off, state, y, theta, 7, 2)
    assert L == pytest.approx(np.mean(Ls), rel=1e-14)
    # per-instance gradient: labels of the other instances do not matter when
    # that instance's weight in the mean is isolated by finite differences of L
    gs = []
    for b in range(len(off) - 1):
        yb = y.copy()
        yb[off[b]:off[b + 1]] = 1.0 - yb[off[b]:off[b + 1]]
        Lb, gb, Lsb = M.batch_loss_and_grad(ops, off, state, yb, theta, 7, 2)
        for c in range(len(off) - 1):
            if c != b:
                assert Lsb[c] == pytest.approx(Ls[c], rel=1e-14)
        gs.append(gb)
    assert np.all(np.isfinite(np.array(gs)))
