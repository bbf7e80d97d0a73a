"""GPU parity of the warm-start network's forward pass, backward pass and
Adam step against the FP64 reference (oracle/mpnn.py), through the C ABI;
parameter files; the layout of the proposal for every replica; and that a few
training steps lower the loss."""
import numpy as np
import pytest

from oracle import mpnn as M
from paper_2412_09285_amd import fem
from paper_2412_09285_amd import workloads as W
from _parity import adam_deviation

pytestmark = pytest.mark.gpu


def small_batch(sizes=(300, 517, 1000), seed0=70_000):
    graphs = [W.batch_instance(b, seed0=seed0, n_override=n) for b, n in enumerate(sizes)]
    off = np.cumsum([0] + [g.n for g in graphs]).astype(np.int64)
    u = np.concatenate([g.u + off[b] for b, g in enumerate(graphs)])
    v = np.concatenate([g.v + off[b] for b, g in enumerate(graphs)])
    w = np.concatenate([g.w for g in graphs])
    parts = [fem.Problem.maxcut(g.n, g.u, g.v, g.w) for g in graphs]
    return graphs, off, M.GraphOps(int(off[-1]), u, v, w), fem.Problem.batch(parts)


def state_of(n, seed, R=None):
    """Fields shaped like a replica part-way through an anneal (|h| ~ 1, some
    beyond the clamp at 8)."""
    rng = np.random.default_rng(seed)
    shape = (n,) if R is None else (n, R)
    return (rng.standard_t(3, size=shape) * 1.5).astype(np.float32)


def test_forward_matches_reference():
    _, off, ops, batch = small_batch()
    theta = W.mpnn_init_weights(5)
    net = fem.MPNN(theta)
    st = state_of(batch.n, 1)
    for draw in (0, 3):
        z = net.forward(batch, st, seed=1234, draw=draw).astype(np.float64)
        zr = M.forward(ops, theta, st, 1234, draw)["z"]
        err = np.abs(z - zr).max() / np.abs(zr).max()
        assert err <= 1e-5, err
    print(f"[mpnn forward] max rel err {err:.2e}", flush=True)


def test_train_step_gradient_and_adam_match_reference():
    _, off, ops, batch = small_batch()
    theta = W.mpnn_init_weights(6)
    st = state_of(batch.n, 2)
    y = np.random.default_rng(2).integers(0, 2, size=int(off[-1])).astype(np.int32)
    net = fem.MPNN(theta)
    lr = 1e-3
    loss, g = net.train_step(batch, st, y, seed=99, draw0=4, lr=lr, want_grad=True)
    Lr, gr, _ = M.batch_loss_and_grad(ops, off, st, y, theta, 99, 4)
    assert loss == pytest.approx(Lr, rel=1e-5)
    rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    mx = np.abs(g - gr).max() / np.abs(gr).max()
    assert rel <= 1e-5 and mx <= 1e-5, (rel, mx)
    # Adam on the master weights: within the deviation the update shows for
    # gradients inside the tested tolerance
    th_ref, _, _ = M.adam_step(theta.astype(np.float64), 0.0, 0.0, gr, 1, lr)

    class P:
        b1, b2, eps, wd = 0.9, 0.999, 1e-8, 0.0
    P.lr = lr
    dev = adam_deviation(theta.astype(np.float64), np.zeros_like(gr), np.zeros_like(gr), gr, 0, P,
                         1e-5 * np.abs(gr).max())
    err = np.abs(net.params().astype(np.float64) - th_ref)
    assert np.all(err <= dev + 1e-6 * np.abs(th_ref).max())
    print(f"[mpnn backward] grad norm rel {rel:.2e}, max rel {mx:.2e}", flush=True)


def test_save_load_and_infer_layout(tmp_path):
    graphs, off, ops, batch = small_batch((200, 333))
    theta = W.mpnn_init_weights(8)
    net = fem.MPNN(theta)
    p = tmp_path / "net.bin"
    net.save(p)
    other = fem.MPNN(np.zeros_like(theta))
    other.load(p)
    assert np.array_equal(other.params(), theta)
    R, alpha = 5, 0.5
    st = state_of(batch.n, 3, R)
    h = other.infer(batch, st, seed=5, alpha=alpha)
    for r in range(R):
        zr = M.forward(ops, theta, st[:, r], 5, r)["z"]
        err = np.abs(h[:, r] / alpha - zr).max() / np.abs(zr).max()
        assert err <= 1e-5, (r, err)


@pytest.mark.parametrize("R", [1, 32, 37])
def test_batched_inference_matches_reference(R):
    """All replicas in one pass (blocks of 32 replicas on the matrix cores,
    a ragged last block at R = 37): every replica's proposal against the FP64
    reference forward of that replica, 1e-5 of its largest logit."""
    graphs, off, ops, batch = small_batch((260, 411))
    theta = W.mpnn_init_weights(14)
    net = fem.MPNN(theta)
    st = state_of(batch.n, 11, R)
    h = net.infer(batch, st, seed=77, alpha=1.0)
    worst = 0.0
    for r in range(R):
        zr = M.forward(ops, theta, st[:, r], 77, r)["z"]
        err = np.abs(h[:, r] - zr).max() / np.abs(zr).max()
        worst = max(worst, err)
    assert worst <= 1e-5, worst
    print(f"[mpnn batched inference R={R}] max rel err {worst:.2e}", flush=True)


def test_batched_inference_of_an_instance_does_not_depend_on_its_batch():
    """Every (node, block of replicas) is formed from its own inputs in a
    fixed order, so the first instance of a batch gets bit-identical
    proposals alone and inside the batch."""
    graphs, off, _, batch = small_batch((301, 517))
    g = graphs[0]
    alone = fem.Problem.maxcut(g.n, g.u, g.v, g.w)
    net = fem.MPNN(W.mpnn_init_weights(22))
    st = state_of(batch.n, 9, 40)
    hb = net.infer(batch, st, seed=3, alpha=1.0)
    ha = net.infer(alone, np.ascontiguousarray(st[:g.n]), seed=3, alpha=1.0)
    assert np.array_equal(hb[:g.n], ha)


def test_infer_on_device_tensors():
    import torch

    _, off, ops, batch = small_batch((250, 400))
    net = fem.MPNN(W.mpnn_init_weights(12))
    st = state_of(batch.n, 4, 6)
    host = net.infer(batch, st, seed=9, alpha=1.5)
    dst = torch.from_numpy(st).cuda()
    out = torch.empty_like(dst)
    net.infer(batch, dst, seed=9, alpha=1.5, out=out)
    assert np.array_equal(out.cpu().numpy(), host)


def test_infer_queued_on_a_stream():
    """fem_mpnn_infer_async: the same proposal, queued on a torch stream
    behind work that writes its input (twice, the second at a smaller R)."""
    import torch

    _, off, ops, batch = small_batch((250, 400))
    net = fem.MPNN(W.mpnn_init_weights(12))
    stream = torch.cuda.Stream()
    for R in (40, 7):
        st = state_of(batch.n, 5 + R, R)
        host = net.infer(batch, st, seed=9, alpha=1.5)
        src = torch.from_numpy(st).cuda()
        with torch.cuda.stream(stream):
            dst = torch.zeros_like(src)
            dst.copy_(src)          # queued on the stream before the inference
            out = torch.empty_like(dst)
        net.infer(batch, dst, seed=9, alpha=1.5, out=out, stream=stream)
        stream.synchronize()
        assert np.array_equal(out.cpu().numpy(), host)


def test_forward_of_an_instance_does_not_depend_on_its_batch():
    """Each node's output is formed from its own inputs in a fixed order
    (layer 2's matrix-core steps included), so the first instance of a batch
    gets bit-identical outputs alone and in the batch (its node indices, and
    so its random features, are the same).  Sizes make the 16-node groups of
    layer 2 straddle the instance boundary."""
    graphs, off, _, batch = small_batch((301, 517, 250))
    g = graphs[0]
    alone = fem.Problem.maxcut(g.n, g.u, g.v, g.w)
    net = fem.MPNN(W.mpnn_init_weights(21))
    st = state_of(batch.n, 8)
    for draw in (0, 5):
        zb = net.forward(batch, st, seed=77, draw=draw)
        za = net.forward(alone, st[: g.n].copy(), seed=77, draw=draw)
        assert np.array_equal(zb[: g.n], za)


def test_training_lowers_the_loss():
    _, off, ops, batch = small_batch((600, 800, 1000, 700))
    st = state_of(batch.n, 5)
    # a label the features determine: the read-out of the state itself
    y = (st > 0).astype(np.int32)
    net = fem.MPNN(W.mpnn_init_weights(9))
    first = net.train_step(batch, st, y, seed=1, draw0=0, lr=3e-3)
    for it in range(60):
        last = net.train_step(batch, st, y, seed=1, draw0=0, lr=3e-3)
    assert last < 0.5 * first
    print(f"[mpnn train] loss {first:.4f} -> {last:.4f}", flush=True)
