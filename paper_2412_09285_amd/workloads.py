"""Seeded synthetic inputs for the Free-Energy Machine (FEM) hot path.

This module is shared by the GPU path, the tests, the benchmark and the oracle
runs.  It draws graphs, CNF formulas and initial fields only: it holds none of
the method's arithmetic (no marginals, energies, gradients or updates), so both
sides of every parity check start from byte-identical inputs.

The paper's benchmark sets (G-set, K2000, Walshaw's partitioning archive,
MaxSAT-2016) are not available here; the recipes below stand in for them with
the shapes, weight distributions and size mixes the paper describes (see
``RECIPES``).  Every generator takes an explicit seed and uses NumPy's PCG64.

Conventions
-----------
* Graphs are undirected edge lists ``(u, v, w)`` with ``u < v``, 0-based node
  ids, no self-loops and no duplicate edges; ``w`` is float32.
* CNF formulas use DIMACS-style signed literals: ``+(v+1)`` for variable ``v``
  and ``-(v+1)`` for its negation, with a clause offset array of length M+1.
* Initial fields ``h0`` are float32, drawn i.i.d. from N(0, std^2), laid out
  node-row / replica-contiguous: ``[N][R]`` for one logit per node (MaxCut,
  Max-k-SAT) and ``[N][R][q]`` for q Potts logits (balanced min-cut).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Graph", "CNF", "rng_for", "er_graph_m", "mpnn_init_weights", "random_sparse_graph", "rgg_3d",
    "random_regular3", "random_ksat", "initial_fields", "batch_instance",
    "RECIPES", "config_graph", "config_cnf", "batch_sizes",
]


@dataclass
class Graph:
    """Undirected weighted graph: each edge {u, v} listed once, u < v."""
    n: int
    u: np.ndarray  # int32 [E]
    v: np.ndarray  # int32 [E]
    w: np.ndarray  # float32 [E]
    meta: dict = field(default_factory=dict)

    @property
    def n_edges(self) -> int:
        return int(self.u.shape[0])

    @property
    def nnz(self) -> int:
        """Directed adjacency entries: every undirected edge counts twice."""
        return 2 * self.n_edges


@dataclass
class CNF:
    """CNF formula with DIMACS-style signed literals (1-based magnitudes)."""
    n_vars: int
    clause_off: np.ndarray  # int64 [M+1]
    lits: np.ndarray        # int32 [clause_off[-1]]
    meta: dict = field(default_factory=dict)

    @property
    def n_clauses(self) -> int:
        return int(self.clause_off.shape[0] - 1)

    @property
    def n_incidences(self) -> int:
        return int(self.lits.shape[0])


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _pair_from_index(n: int, k: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Map k in [0, n(n-1)/2) to the k-th pair (i, j), i < j, row-major."""
    k = k.astype(np.int64)
    # row i starts at s(i) = i*n - i*(i+1)/2 ; find the largest i with s(i) <= k
    i = np.floor((2 * n - 1 - np.sqrt((2.0 * n - 1) ** 2 - 8.0 * k)) / 2).astype(np.int64)
    s = i * n - i * (i + 1) // 2
    # fix floating-point off-by-one in either direction
    over = s > k
    i[over] -= 1
    s = i * n - i * (i + 1) // 2
    nxt = (i + 1) * n - (i + 1) * (i + 2) // 2
    under = nxt <= k
    i[under] += 1
    s = i * n - i * (i + 1) // 2
    j = k - s + i + 1
    return i.astype(np.int32), j.astype(np.int32)


def er_graph_m(n: int, m: int, seed: int, weights: str = "one") -> Graph:
    """Erdos-Renyi G(n, m): m distinct pairs drawn uniformly without replacement
    from all n(n-1)/2 pairs.  ``weights`` is "one" (all +1) or "pm1" (+1/-1
    with equal probability)."""
    rng = rng_for(seed)
    total = n * (n - 1) // 2
    if m > total:
        raise ValueError("too many edges for G(n, m)")
    if total <= 50_000_000:
        k = np.sort(rng.choice(total, size=m, replace=False))
    else:  # sparse regime: rejection on pair ids
        picked: set[int] = set()
        ks = []
        while len(ks) < m:
            cand = rng.integers(0, total, size=2 * (m - len(ks)) + 16)
            for c in cand.tolist():
                if c not in picked:
                    picked.add(c)
                    ks.append(c)
                    if len(ks) == m:
                        break
        k = np.sort(np.asarray(ks, dtype=np.int64))
    u, v = _pair_from_index(n, k)
    w = _draw_weights(rng, m, weights)
    return Graph(n, u, v, w, {"kind": "er_m", "seed": seed})


def _draw_weights(rng: np.random.Generator, m: int, weights: str) -> np.ndarray:
    if weights == "one":
        return np.ones(m, dtype=np.float32)
    if weights == "pm1":
        return np.where(rng.integers(0, 2, size=m) == 1, 1.0, -1.0).astype(np.float32)
    raise ValueError(weights)


def random_sparse_graph(n: int, n_edges: int, seed: int, weights: str = "pm1") -> Graph:
    """Endpoints drawn uniformly; self-loops and duplicate pairs rejected until
    exactly ``n_edges`` distinct edges exist (the first occurrence of a pair in
    draw order is kept)."""
    rng = rng_for(seed)
    keys = np.empty(0, dtype=np.int64)
    order = np.empty(0, dtype=np.int64)
    drawn = 0
    while keys.shape[0] < n_edges:
        need = n_edges - keys.shape[0]
        a = rng.integers(0, n, size=int(need * 1.2) + 64)
        b = rng.integers(0, n, size=a.shape[0])
        ok = a != b
        a, b = a[ok], b[ok]
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        new_keys = lo.astype(np.int64) * n + hi
        new_order = drawn + np.arange(new_keys.shape[0], dtype=np.int64)
        drawn += new_keys.shape[0]
        allk = np.concatenate([keys, new_keys])
        allo = np.concatenate([order, new_order])
        uk, first = np.unique(allk, return_index=True)
        # keep the earliest n_edges distinct pairs in draw order
        sel = np.argsort(allo[first], kind="stable")[:n_edges]
        keys, order = uk[sel], allo[first][sel]
    srt = np.argsort(order, kind="stable")
    keys = keys[srt]
    u = (keys // n).astype(np.int32)
    v = (keys % n).astype(np.int32)
    w = _draw_weights(rng, n_edges, weights)
    return Graph(n, u, v, w, {"kind": "uniform_endpoints", "seed": seed})


def rgg_radius_for_degree(n: int, mean_degree: float) -> float:
    """Radius r solving (n-1) * [(4/3) pi r^3 - (3/2) pi r^4] = mean_degree,
    the expected degree in the unit cube with the first-order boundary loss."""
    lo, hi = 0.0, 0.5
    for _ in range(200):
        r = 0.5 * (lo + hi)
        f = (n - 1) * ((4.0 / 3.0) * math.pi * r ** 3 - 1.5 * math.pi * r ** 4)
        if f < mean_degree:
            lo = r
        else:
            hi = r
    return 0.5 * (lo + hi)


def rgg_3d(n: int, mean_degree: float, seed: int) -> Graph:
    """3-D random geometric graph: n points uniform in [0,1)^3, an edge for
    every pair closer than r (Euclidean), unit weights.  Node order is the
    draw order (no spatial sorting)."""
    from scipy.spatial import cKDTree

    rng = rng_for(seed)
    pts = rng.random((n, 3))
    r = rgg_radius_for_degree(n, mean_degree)
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
    pairs = np.sort(pairs, axis=1)
    order = np.lexsort((pairs[:, 1], pairs[:, 0]))
    pairs = pairs[order]
    u = pairs[:, 0].astype(np.int32)
    v = pairs[:, 1].astype(np.int32)
    w = np.ones(u.shape[0], dtype=np.float32)
    return Graph(n, u, v, w, {"kind": "rgg3d", "seed": seed, "radius": r,
                              "realised_mean_degree": 2.0 * u.shape[0] / n})


def random_regular3(n: int, seed: int, weights: str = "pm1") -> Graph:
    """Random 3-regular simple graph by the pairing (configuration) model with
    restarts; n is rounded up to even."""
    if n % 2:
        n += 1
    rng = rng_for(seed)
    for attempt in range(1000):
        stubs = np.repeat(np.arange(n, dtype=np.int64), 3)
        rng.shuffle(stubs)
        a, b = stubs[0::2], stubs[1::2]
        if np.any(a == b):
            continue
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        key = lo * n + hi
        if np.unique(key).shape[0] != key.shape[0]:
            continue
        key = np.sort(key)
        u = (key // n).astype(np.int32)
        v = (key % n).astype(np.int32)
        w = _draw_weights(rng, u.shape[0], weights)
        return Graph(n, u, v, w, {"kind": "regular3", "seed": seed, "attempts": attempt + 1})
    raise RuntimeError("pairing model failed to produce a simple graph")


def random_ksat(n_vars: int, n_clauses: int, k: int, seed: int) -> CNF:
    """Random k-SAT: each clause has k distinct variables drawn uniformly and
    independent fair signs."""
    rng = rng_for(seed)
    # k distinct variables per clause: draw, then redraw rows with repeats
    var = rng.integers(0, n_vars, size=(n_clauses, k))
    while True:
        srt = np.sort(var, axis=1)
        bad = np.any(srt[:, 1:] == srt[:, :-1], axis=1) if k > 1 else np.zeros(n_clauses, bool)
        nb = int(bad.sum())
        if nb == 0:
            break
        var[bad] = rng.integers(0, n_vars, size=(nb, k))
    sign = rng.integers(0, 2, size=(n_clauses, k))
    lits = np.where(sign == 1, var + 1, -(var + 1)).astype(np.int32).reshape(-1)
    off = np.arange(0, (n_clauses + 1) * k, k, dtype=np.int64)
    return CNF(n_vars, off, lits, {"kind": "random_ksat", "k": k, "seed": seed})


def mpnn_init_weights(seed: int) -> np.ndarray:
    """Initial parameters of the warm-start network, float32, as one flat
    vector in the order A1 [8][64], B1 [8][64], b1 [64], A2 [64][64],
    B2 [64][64], b2 [64], c [64], d [1]: matrices uniform in
    +/- 1/sqrt(fan_in), biases zero."""
    rng = rng_for(seed)
    parts = []
    for fan_in, shape in ((8, (8, 64)), (8, (8, 64)), (None, (64,)), (64, (64, 64)), (64, (64, 64)),
                          (None, (64,)), (64, (64,)), (None, (1,))):
        if fan_in is None:
            parts.append(np.zeros(shape))
        else:
            b = 1.0 / math.sqrt(fan_in)
            parts.append(rng.uniform(-b, b, size=shape))
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)


def initial_fields(n: int, R: int, seed: int, q: int = 1, std: float = 0.01) -> np.ndarray:
    """h0 ~ N(0, std^2) i.i.d., float32, shape [n, R] (q == 1) or [n, R, q]."""
    rng = rng_for(seed)
    shape = (n, R) if q == 1 else (n, R, q)
    return (rng.standard_normal(size=shape) * std).astype(np.float32)


# ---------------------------------------------------------------------------
# The five workload recipes.  Seeds: graph seed = recipe number, h0 seed =
# 100 + recipe number; batched instance b uses seed 50000 + b, training
# instances 60000 + j, and their h0 seed is 1000000 + the instance seed.
# ---------------------------------------------------------------------------
RECIPES = {
    1: dict(name="maxcut_er800", problem="maxcut", n=800, edges=19_176, R=16, T=500,
            weights="one", beta=(0.01, 5.0), lr=0.1, dtype="f32"),
    2: dict(name="maxcut_sparse1e5", problem="maxcut", n=100_000, edges=300_000, R=256,
            T=2000, weights="pm1", beta=(0.01, 5.0), lr=0.1, dtype="f32"),
    3: dict(name="bmincut_rgg1e6_q8", problem="bmincut", n=1_000_000, mean_degree=14.0,
            q=8, lam=1.0, R=16, T=3000, beta=(0.01, 5.0), lr=0.1, dtype="bf16"),
    4: dict(name="max3sat_1e5", problem="maxsat", n=100_000, clauses=800_000, k=3, R=64,
            T=2000, beta=(0.01, 5.0), lr=0.1, dtype="f32"),
    5: dict(name="batch512_maxcut", problem="maxcut_batch", instances=512,
            n_range=(1_000, 50_000), R=32, beta=(0.01, 5.0), lr=0.1, dtype="bf16"),
}


def config_graph(cfg: int, n: int | None = None) -> Graph:
    """The graph of recipe ``cfg`` (1, 2 or 3).  ``n`` shrinks the node count
    (same recipe, same density) for quick parity runs."""
    rc = RECIPES[cfg]
    if cfg == 1:
        nn = rc["n"] if n is None else n
        m = rc["edges"] if n is None else int(round(rc["edges"] * nn * (nn - 1) / (rc["n"] * (rc["n"] - 1))))
        return er_graph_m(nn, m, seed=cfg, weights=rc["weights"])
    if cfg == 2:
        nn = rc["n"] if n is None else n
        m = rc["edges"] if n is None else 3 * nn
        return random_sparse_graph(nn, m, seed=cfg, weights=rc["weights"])
    if cfg == 3:
        nn = rc["n"] if n is None else n
        return rgg_3d(nn, rc["mean_degree"], seed=cfg)
    raise ValueError(cfg)


def config_cnf(cfg: int = 4, n: int | None = None) -> CNF:
    rc = RECIPES[cfg]
    nn = rc["n"] if n is None else n
    m = rc["clauses"] if n is None else 8 * nn
    return random_ksat(nn, m, rc["k"], seed=cfg)


def batch_sizes(n_inst: int = 512, seed0: int = 50_000, n_range=(1_000, 50_000)) -> list[int]:
    """Instance sizes: N_b = round(exp(U[ln lo, ln hi])) with seed seed0 + b."""
    out = []
    lo, hi = math.log(n_range[0]), math.log(n_range[1])
    for b in range(n_inst):
        rng = rng_for(seed0 + b)
        out.append(int(round(math.exp(rng.uniform(lo, hi)))))
    return out


def batch_instance(b: int, seed0: int = 50_000, n_range=(1_000, 50_000), n_override: int | None = None) -> Graph:
    """Instance b of the batched workload: even b -> random 3-regular, odd b ->
    Erdos-Renyi G(n, 5n) (mean degree 10), weights +1/-1."""
    seed = seed0 + b
    rng = rng_for(seed)
    lo, hi = math.log(n_range[0]), math.log(n_range[1])
    n = int(round(math.exp(rng.uniform(lo, hi)))) if n_override is None else n_override
    if b % 2 == 0:
        g = random_regular3(n, seed=seed + 7_000_000, weights="pm1")
    else:
        g = random_sparse_graph(n, 5 * n, seed=seed + 7_000_000, weights="pm1")
    g.meta.update({"instance": b, "seed": seed})
    return g


def community_sizes(n: int, seed: int, mean: float = 4.0) -> np.ndarray:
    """Node weights of a coarsened graph (each coarse node stands for a
    community of original nodes): V_i >= 1, geometric with the given mean,
    int32."""
    rng = rng_for(seed)
    return rng.geometric(1.0 / mean, size=n).astype(np.int32)


def complete_pm1(n: int, seed: int) -> Graph:
    """Complete graph K_n with independent +1/-1 weights of equal probability
    (the shape of the K2000 MaxCut benchmark: all-to-all, unit magnitudes)."""
    rng = rng_for(seed)
    iu, ju = np.triu_indices(n, k=1)
    w = _draw_weights(rng, iu.shape[0], "pm1")
    return Graph(n, iu.astype(np.int32), ju.astype(np.int32), w, {"kind": "complete_pm1", "seed": seed})


def dense_matrix(g: Graph) -> np.ndarray:
    """Symmetric float32 [n][n] weight matrix of an edge list (zero diagonal)."""
    W = np.zeros((g.n, g.n), dtype=np.float32)
    W[g.u, g.v] = g.w
    W[g.v, g.u] = g.w
    return W
