"""FP64 reference of the message-passing warm-start network (test infrastructure
only; the product path never imports it).

The paper has no neural network: this is the learned warm start built on top
of FEM.  It maps the state of one replica part-way through an anneal to a
proposal for that replica's final read-out, from which a shorter anneal
continues.  Its specification, which the HIP kernels implement independently:

* Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
  "Parallel random numbers: as easy as 1, 2, 3", SC 2011), written here from
  that definition; uniforms in [-1, 1) from the top 24 bits of a Philox word,
  so they are exact in float32 and float64 alike.
* Node features x_i (8) from one replica's fields s (float32, length n):
  [1, ln(1 + deg_i), mean_{j in N(i)} W_ij (0 if isolated), tanh(s_i / 2),
  clamp(s_i / 4, -2, 2), u_i^1, u_i^2, u_i^3] with u words 0..2 of
  Philox(counter = (i, draw, 0, 0), key = (seed mod 2^32, seed div 2^32)).
* Two layers, width 64, mean aggregation a_i = (1 / max(deg_i, 1)) sum_j W_ij v_j:
      pre1 = x A1 + a1(x) B1 + b1,      H1 = relu(pre1)
      pre2 = H1 A2 + a2(H1) B2 + b2,    H2 = relu(pre2)
      z = H2 c + d                      (one logit per node)
  with every weight rounded to bfloat16 (round to nearest even) before use.
* Loss of a batch of instances (a block-diagonal union), each with its own
  replica's fields and label y (0/1 per node, the final read-out of that
  replica): the mean over instances of BCE(z, y) = mean_i [softplus(z_i) -
  y_i z_i].
* Flat parameter vector (9409 values): A1 [8][64], B1 [8][64], b1 [64],
  A2 [64][64], B2 [64][64], b2 [64], c [64], d [1].

Pinned by central finite differences of the loss (tests/test_mpnn_oracle.py)
and by the Philox known-answer vectors (tests/golden/philox_kat.json).
"""
from __future__ import annotations

import numpy as np

D_IN, HID = 8, 64
SHAPES = [("A1", (D_IN, HID)), ("B1", (D_IN, HID)), ("b1", (HID,)), ("A2", (HID, HID)), ("B2", (HID, HID)),
          ("b2", (HID,)), ("c", (HID,)), ("d", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32 with 10 rounds.  Counters are uint32 arrays (any
    broadcastable shape), the key two Python ints.  Returns four uint32
    arrays."""
    c = [np.asarray(x, dtype=np.uint64) & _MASK for x in (c0, c1, c2, c3)]
    k0, k1 = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & 0xFFFFFFFF
            k1 = (k1 + _W1) & 0xFFFFFFFF
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
    return [x.astype(np.uint32) for x in c]


def uniform_pm1(word):
    """uint32 -> [-1, 1): top 24 bits scaled by 2^-23, minus one (exact)."""
    return (np.asarray(word, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) * 2.0 ** -23 - 1.0


def bf16_round(w):
    """Round float32 values to bfloat16 (round to nearest, ties to even) and
    return them as float64."""
    f = np.ascontiguousarray(w, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta):
    out, k = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[k:k + n], dtype=np.float64).reshape(shp)
        k += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


class GraphOps:
    """Mean aggregation over a graph given as an undirected edge list."""

    def __init__(self, n, u, v, w):
        import scipy.sparse as sp

        u = np.asarray(u, dtype=np.int64)
        v = np.asarray(v, dtype=np.int64)
        w = np.asarray(w, dtype=np.float64)
        self.n = n
        self.W = sp.csr_matrix((np.concatenate([w, w]), (np.concatenate([u, v]), np.concatenate([v, u]))),
                               shape=(n, n))
        self.deg = np.bincount(np.concatenate([u, v]), minlength=n).astype(np.float64)
        wsum = np.asarray(self.W.sum(axis=1)).reshape(-1)
        self.wmean = np.where(self.deg > 0, wsum / np.maximum(self.deg, 1.0), 0.0)
        self.inv = 1.0 / np.maximum(self.deg, 1.0)

    def agg(self, V):
        """a_i = (1 / max(deg_i, 1)) sum_j W_ij V_j"""
        return self.inv[:, None] * (self.W @ V)

    def agg_T(self, G):
        """adjoint of agg: dV_j = sum_i W_ij G_i / max(deg_i, 1)"""
        return self.W.T @ (self.inv[:, None] * G)


def features(ops: GraphOps, state, seed: int, draw: int):
    n = ops.n
    st = np.asarray(state, dtype=np.float64).reshape(n)
    i = np.arange(n, dtype=np.uint64)
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    r0 = philox4x32_10(i, np.uint64(draw), 0, 0, k0, k1)
    x = np.empty((n, D_IN))
    x[:, 0] = 1.0
    x[:, 1] = np.log1p(ops.deg)
    x[:, 2] = ops.wmean
    x[:, 3] = np.tanh(st / 2.0)
    x[:, 4] = np.clip(st / 4.0, -2.0, 2.0)
    x[:, 5] = uniform_pm1(r0[0])
    x[:, 6] = uniform_pm1(r0[1])
    x[:, 7] = uniform_pm1(r0[2])
    return x


def forward(ops: GraphOps, theta, state, seed: int, draw: int, quantize: bool = True):
    """quantize=False skips the bfloat16 rounding (used to check the backward
    pass by finite differences, where the rounding would hide the steps)."""
    P = unpack(bf16_round(np.asarray(theta, dtype=np.float32)) if quantize else np.asarray(theta, dtype=np.float64))
    x = features(ops, state, seed, draw)
    a1 = ops.agg(x)
    pre1 = x @ P["A1"] + a1 @ P["B1"] + P["b1"]
    H1 = np.maximum(pre1, 0.0)
    a2 = ops.agg(H1)
    pre2 = H1 @ P["A2"] + a2 @ P["B2"] + P["b2"]
    H2 = np.maximum(pre2, 0.0)
    z = H2 @ P["c"] + P["d"][0]
    return dict(x=x, a1=a1, pre1=pre1, H1=H1, a2=a2, pre2=pre2, H2=H2, z=z, P=P)


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def bce(z, y):
    """mean_i softplus(z_i) - y_i z_i"""
    return float(np.mean(softplus(z) - y * z))


def batch_loss_and_grad(ops: GraphOps, inst_off, state, labels, theta, seed: int, draw: int,
                        quantize: bool = True):
    """Loss and gradient of one training step on a block-diagonal batch: one
    forward over the union graph (features keyed by the node's index in the
    union), BCE per instance, mean over the instances.  Returns (loss, grad,
    per-instance losses)."""
    f = forward(ops, theta, state, seed, draw, quantize)
    P = f["P"]
    z = f["z"]
    y = np.asarray(labels, dtype=np.float64)
    B = len(inst_off) - 1
    dz = np.zeros_like(z)
    Ls = []
    for b in range(B):
        sl = slice(inst_off[b], inst_off[b + 1])
        nb = inst_off[b + 1] - inst_off[b]
        Ls.append(bce(z[sl], y[sl]))
        dz[sl] = (1.0 / (1.0 + np.exp(-z[sl])) - y[sl]) / nb / B
    grads = {}
    grads["c"] = f["H2"].T @ dz
    grads["d"] = np.array([dz.sum()])
    dpre2 = np.outer(dz, P["c"]) * (f["pre2"] > 0)
    grads["A2"] = f["H1"].T @ dpre2
    grads["B2"] = f["a2"].T @ dpre2
    grads["b2"] = dpre2.sum(0)
    dH1 = dpre2 @ P["A2"].T + ops.agg_T(dpre2 @ P["B2"].T)
    dpre1 = dH1 * (f["pre1"] > 0)
    grads["A1"] = f["x"].T @ dpre1
    grads["B1"] = f["a1"].T @ dpre1
    grads["b1"] = dpre1.sum(0)
    return float(np.mean(Ls)), pack(grads), Ls


def batch_loss(ops: GraphOps, inst_off, state, labels, theta, seed: int, draw: int, quantize: bool = True):
    z = forward(ops, theta, state, seed, draw, quantize)["z"]
    y = np.asarray(labels, dtype=np.float64)
    return float(np.mean([bce(z[inst_off[b]:inst_off[b + 1]], y[inst_off[b]:inst_off[b + 1]])
                          for b in range(len(inst_off) - 1)]))


def adam_step(theta, m1, m2, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """torch.optim.Adam step t (1-based) on float64 copies; returns new arrays."""
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    th = theta - (lr / (1 - b1 ** t)) * m1 / (np.sqrt(m2) / np.sqrt(1 - b2 ** t) + eps)
    return th, m1, m2
