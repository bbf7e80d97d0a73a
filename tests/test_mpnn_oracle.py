"""Pins of the FP64 reference of the warm-start network: the Philox generator
against its published known-answer vectors, bfloat16 rounding against its
definition, the analytic backward pass against central finite differences of
the loss, and the flip invariance of the loss."""
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


def test_uniform_features_range_and_exactness():
    ops = M.GraphOps(50, np.array([0, 1]), np.array([1, 2]), np.array([1.0, -1.0]))
    x = M.features(ops, seed=123, draw=4)
    assert np.all(x[:, 0] == 1.0)
    assert np.all((x[:, 3:] >= -1) & (x[:, 3:] < 1))
    assert np.array_equal(x[:, 3:].astype(np.float32).astype(np.float64), x[:, 3:])
    assert x[0, 2] == 1.0 and x[1, 2] == 0.0 and x[3, 2] == 0.0


@pytest.fixture(scope="module")
def small_items():
    items = []
    for b in range(3):
        g = W.random_sparse_graph(40 + 7 * b, 90 + 10 * b, seed=b, weights="pm1")
        y = np.random.default_rng(b).integers(0, 2, size=g.n).astype(np.float64)
        items.append((M.GraphOps(g.n, g.u, g.v, g.w), y))
    return items


def test_backward_matches_finite_differences(small_items):
    theta = W.mpnn_init_weights(7).astype(np.float64)
    draws = [0, 3, 5]
    L, grad = M.loss_and_grad(small_items, theta, 99, draws, quantize=False)
    assert L == pytest.approx(M.loss_only(small_items, theta, 99, draws, quantize=False), rel=1e-14)
    rng = np.random.default_rng(1)
    eps = 1e-6
    # every parameter block, a few coordinates each
    idx = []
    k = 0
    for name, shp in M.SHAPES:
        n = int(np.prod(shp))
        idx += list(k + rng.choice(n, size=min(n, 6), replace=False))
        k += n
    for j in idx:
        tp = theta.copy(); tp[j] += eps
        tm = theta.copy(); tm[j] -= eps
        fd = (M.loss_only(small_items, tp, 99, draws, False) - M.loss_only(small_items, tm, 99, draws, False)) / (2 * eps)
        assert abs(fd - grad[j]) <= 1e-6 * max(1.0, abs(grad).max()), (j, fd, grad[j])
    # directional derivative
    dv = rng.normal(size=theta.size)
    e2 = 1e-6
    fd = (M.loss_only(small_items, theta + e2 * dv, 99, draws, False)
          - M.loss_only(small_items, theta - e2 * dv, 99, draws, False)) / (2 * e2)
    assert fd == pytest.approx(float(grad @ dv), rel=1e-6, abs=1e-9)


def test_loss_is_flip_invariant(small_items):
    theta = W.mpnn_init_weights(3).astype(np.float64)
    flipped = [(ops, 1.0 - y) for ops, y in small_items]
    a = M.loss_only(small_items, theta, 5, [0, 1, 2])
    b = M.loss_only(flipped, theta, 5, [0, 1, 2])
    assert a == pytest.approx(b, rel=1e-15)


def test_batch_loss_matches_per_instance_definition():
    """On a block-diagonal union the batch loss equals the mean of the
    per-instance losses computed on the union's forward pass, and its
    gradient matches finite differences."""
    gs = [W.random_sparse_graph(30 + 5 * b, 70, seed=10 + b, weights="pm1") for b in range(3)]
    off = np.cumsum([0] + [g.n for g in gs])
    u = np.concatenate([g.u + off[b] for b, g in enumerate(gs)])
    v = np.concatenate([g.v + off[b] for b, g in enumerate(gs)])
    w = np.concatenate([g.w for g in gs])
    ops = M.GraphOps(int(off[-1]), u, v, w)
    y = np.random.default_rng(4).integers(0, 2, size=int(off[-1])).astype(np.float64)
    theta = W.mpnn_init_weights(11).astype(np.float64)
    L, grad, Ls = M.batch_loss_and_grad(ops, off, y, theta, 7, 2, quantize=False)
    assert L == pytest.approx(np.mean([min(a, b) for a, b in Ls]), rel=1e-14)
    rng = np.random.default_rng(0)
    for j in rng.choice(theta.size, size=20, replace=False):
        tp = theta.copy(); tp[j] += 1e-6
        tm = theta.copy(); tm[j] -= 1e-6
        fd = (M.batch_loss_and_grad(ops, off, y, tp, 7, 2, False)[0]
              - M.batch_loss_and_grad(ops, off, y, tm, 7, 2, False)[0]) / 2e-6
        assert abs(fd - grad[j]) <= 1e-6 * max(1.0, np.abs(grad).max())
