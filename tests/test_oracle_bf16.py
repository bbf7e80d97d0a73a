"""Pins of the oracle's bfloat16-copy mode (neighbours read a bfloat16 copy
of the marginals; everything else in double).

* The rounding itself: every result is a bfloat16 value, the nearest one to
  the input, ties to the even neighbour; brute force over the neighbouring
  bfloat16 values, exact midpoints, and torch's float32 -> bfloat16
  conversion on float32 inputs.
* Where every stored value is already a bfloat16 number the mode changes
  nothing: fields chosen so that m = tanh(h/2) (MaxCut), P = softmax(h)
  (Potts) or min(P, 1 - P) (Max-k-SAT) are bfloat16 values give the FP64
  gradient and energies to rounding error.
* What is never rounded: the entropy, and a unit clause (no other literal to
  read) gives the FP64 gradient and energy for any fields.
* The change against FP64 is bounded by the rounding of the gathered values
  and is not zero.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2412_09285_amd import workloads as W


def _bf16_grid_neighbours(x):
    """The bfloat16 values around x (brute-force candidates): the bfloat16
    patterns within two steps of float32(x)'s upper half."""
    b = np.array([x], dtype=np.float32).view(np.uint32)[0] >> 16
    out = []
    for d in range(-2, 3):
        pat = (int(b) + d) & 0xffff
        v = np.array([pat << 16], dtype=np.uint32).view(np.float32)[0]
        if np.isfinite(v):
            out.append((float(v), pat))
    return out


def test_round_bf16_is_the_nearest_bf16_value_ties_to_even():
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.uniform(-1, 1, 3000), 10.0 ** rng.uniform(-40, 3, 3000) * rng.choice([-1, 1], 3000)])
    for x in xs:
        r = orc.round_bf16(x)
        cands = _bf16_grid_neighbours(x)
        best = min(abs(v - x) for v, _ in cands)
        near = [(v, p) for v, p in cands if abs(v - x) == best]
        if len(near) == 1:
            assert r == near[0][0], (x, r, near)
        else:
            even = [v for v, p in near if p % 2 == 0]
            assert r == even[0], (x, r, near)


def test_round_bf16_exact_midpoints_go_to_the_even_neighbour():
    # 1 + 2^-8 lies halfway between 1 (even pattern) and 1 + 2^-7 (odd)
    assert orc.round_bf16(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3 * 2^-8 lies halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert orc.round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert orc.round_bf16(-(1.0 + 2.0 ** -8)) == -1.0
    # just above a midpoint rounds up
    assert orc.round_bf16(1.0 + 2.0 ** -8 + 2.0 ** -40) == 1.0 + 2.0 ** -7
    assert orc.round_bf16(0.0) == 0.0


def test_round_bf16_matches_torch_on_float32_inputs():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(5000), rng.uniform(-1, 1, 5000) * 1e-30]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([orc.round_bf16(float(v)) for v in x])
    assert np.array_equal(got, ref)


def _bf16_values(rng, shape, lo, hi):
    v = rng.uniform(lo, hi, shape)
    return np.vectorize(orc.round_bf16)(v)


def test_maxcut_mode_is_exact_on_bf16_marginals():
    g = W.random_sparse_graph(40, 120, seed=3, weights="pm1")
    rng = np.random.default_rng(4)
    m = _bf16_values(rng, (40, 5), -0.999, 0.999)
    h = 2.0 * np.arctanh(m)
    a = orc.maxcut_grad(40, g.u, g.v, g.w, h, 0.7)
    b = orc.maxcut_grad(40, g.u, g.v, g.w, h, 0.7, mdt=1)
    for x, y in zip(a, b):
        assert np.allclose(x, y, rtol=1e-12, atol=1e-12)


def test_potts_mode_is_exact_on_bf16_marginals():
    g = W.random_sparse_graph(30, 90, seed=5, weights="one")
    q, R = 4, 3
    rng = np.random.default_rng(6)
    # rows of four bfloat16 probabilities summing to 1 exactly
    rows = np.array([[0.5, 0.25, 0.125, 0.125], [0.75, 0.125, 0.0625, 0.0625], [0.375, 0.375, 0.1875, 0.0625]])
    P = rows[rng.integers(0, 3, size=(30, R))]
    P = np.take_along_axis(P, np.argsort(rng.random((30, R, q)), axis=2), axis=2)
    h = np.log(P) + rng.standard_normal((30, R, 1))     # a per-row shift leaves the softmax unchanged
    a = orc.bmincut_grad(30, g.u, g.v, g.w, q, 0.4, h, 0.9)
    b = orc.bmincut_grad(30, g.u, g.v, g.w, q, 0.4, h, 0.9, mdt=1)
    for x, y in zip(a, b):
        assert np.allclose(x, y, rtol=1e-12, atol=1e-12)


def test_maxsat_mode_is_exact_on_bf16_marginals():
    cnf = W.random_ksat(30, 100, 3, seed=7)
    rng = np.random.default_rng(8)
    small = _bf16_values(rng, (30, 4), 1e-4, 0.5)
    sign = rng.choice([-1.0, 1.0], size=(30, 4))
    h = sign * np.log((1.0 - small) / small)               # min(P, 1 - P) = small
    a = orc.maxsat_grad(30, cnf.clause_off, cnf.lits, h, 0.8)
    b = orc.maxsat_grad(30, cnf.clause_off, cnf.lits, h, 0.8, mdt=1)
    for x, y in zip(a, b):
        assert np.allclose(x, y, rtol=1e-12, atol=1e-12)


def test_entropy_and_unit_clauses_are_never_rounded():
    rng = np.random.default_rng(9)
    g = W.random_sparse_graph(40, 120, seed=3, weights="pm1")
    h = rng.standard_normal((40, 6)) * 2
    _, _, Sa = orc.maxcut_grad(40, g.u, g.v, g.w, h, 0.7)
    _, _, Sb = orc.maxcut_grad(40, g.u, g.v, g.w, h, 0.7, mdt=1)
    assert np.array_equal(Sa, Sb)
    # unit clauses: no other literal is read, so nothing is rounded
    lits = np.array([1, -2, 3, 3, -1], dtype=np.int32)
    off = np.arange(6, dtype=np.int64)
    h3 = rng.standard_normal((3, 4)) * 3
    a = orc.maxsat_grad(3, off, lits, h3, 0.5)
    b = orc.maxsat_grad(3, off, lits, h3, 0.5, mdt=1)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_change_is_within_the_rounding_of_the_gathered_values():
    """MaxCut: each gathered m_j moves by at most 2^-9 |m_j| (8 significant
    bits, round to nearest), so |dg_i| <= P(1-P) 2 sum_j |W_ij| 2^-9 |m_j| and
    |dU| <= 2^-9 sum over edges |W_ij| |m_i m_j|; the change is not zero."""
    g = W.random_sparse_graph(60, 240, seed=11, weights="pm1")
    rng = np.random.default_rng(12)
    h = rng.standard_normal((60, 4)) * 1.5
    ga, Ua, _ = orc.maxcut_grad(60, g.u, g.v, g.w, h, 0.9)
    gb, Ub, _ = orc.maxcut_grad(60, g.u, g.v, g.w, h, 0.9, mdt=1)
    m = np.tanh(h / 2)
    p = 1 / (1 + np.exp(-h))
    s = np.zeros_like(h)
    np.add.at(s, g.u, np.abs(g.w)[:, None] * np.abs(m[g.v]))
    np.add.at(s, g.v, np.abs(g.w)[:, None] * np.abs(m[g.u]))
    bound = p * (1 - p) * 2 * 2.0 ** -9 * s + 1e-12
    assert np.all(np.abs(gb - ga) <= bound)
    assert np.abs(gb - ga).max() > 0
    ubound = 2.0 ** -9 * np.sum(np.abs(g.w)[:, None] * np.abs(m[g.u] * m[g.v]), axis=0) + 1e-12
    assert np.all(np.abs(Ub - Ua) <= ubound)
