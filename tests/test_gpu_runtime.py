"""GPU runtime properties: graph replay equals eager stepping, checkpoints
resume bit for bit, runs are deterministic, every launch shape gives the same
fields, a batch of instances equals the instances run alone, replicas are
independent, and the error states of the C ABI."""
import numpy as np
import pytest
import torch

from paper_2412_09285_amd import fem
from paper_2412_09285_amd import workloads as W

pytestmark = pytest.mark.gpu


def maxcut_problem(n=1200, seed=3):
    g = W.random_sparse_graph(n, 3 * n, seed=seed, weights="pm1")
    return g, fem.Problem.maxcut(g.n, g.u, g.v, g.w)


def run_fields(prob, h0, R, steps, T=200, tile=None, stream=None, graph=False, **kw):
    s = fem.Solver(prob, fem.default_params(replicas=R, steps=T, **kw), stream=stream)
    if tile is not None:
        s.set_tile(*tile)
    s.set_fields(h0)
    if graph:
        s.run_until(steps)
    else:
        s.step(steps)
    return s.fields(), s


def test_graph_equals_eager_and_replays():
    g, prob = maxcut_problem()
    R = 64
    h0 = W.initial_fields(g.n, R, seed=1)
    st = torch.cuda.Stream()
    he, se = run_fields(prob, h0, R, 80, stream=st, eval_every=20, record_energies=1)
    hg, sg = run_fields(prob, h0, R, 80, stream=st, graph=True, eval_every=20, record_energies=1)
    assert np.array_equal(he, hg)
    assert np.array_equal(se.energy_history(0, 80)[0], sg.energy_history(0, 80)[0])
    assert np.array_equal(se.anytime_best(), sg.anytime_best())
    # replay the cached graph three times, with eager work in between
    for _ in range(3):
        sg.set_fields(h0)
        sg.step(0)
        sg.run_until(80)
        assert np.array_equal(sg.fields(), he)


def test_graph_equals_eager_potts():
    g = W.rgg_3d(700, 12.0, seed=2)
    prob = fem.Problem.bmincut(g.n, g.u, g.v, g.w, 4)
    R = 16
    h0 = W.initial_fields(g.n, R, seed=2, q=4)
    st = torch.cuda.Stream()
    he, _ = run_fields(prob, h0, R, 50, stream=st, lam=0.5)
    hg, _ = run_fields(prob, h0, R, 50, stream=st, graph=True, lam=0.5)
    assert np.array_equal(he, hg)


@pytest.mark.parametrize("kind", ["maxcut", "bmincut", "maxsat"])
def test_checkpoint_resume_bitexact(kind):
    R = 32
    if kind == "maxcut":
        g, prob = maxcut_problem()
        h0 = W.initial_fields(g.n, R, seed=5)
        kw = {}
    elif kind == "bmincut":
        g = W.rgg_3d(500, 10.0, seed=5)
        prob = fem.Problem.bmincut(g.n, g.u, g.v, g.w, 8)
        h0 = W.initial_fields(g.n, R, seed=5, q=8)
        kw = {"lam": 0.7, "lambda_ramp": 1}
    else:
        cnf = W.random_ksat(800, 6400, 3, seed=5)
        prob = fem.Problem.maxsat(cnf.n_vars, cnf.clause_off, cnf.lits)
        h0 = W.initial_fields(cnf.n_vars, R, seed=5)
        kw = {}
    straight, _ = run_fields(prob, h0, R, 60, T=100, **kw)
    s1 = fem.Solver(prob, fem.default_params(replicas=R, steps=100, **kw))
    s1.set_fields(h0)
    s1.step(25)
    blob = s1.get_state()
    s1.close()
    s2 = fem.Solver(prob, fem.default_params(replicas=R, steps=100, **kw))
    s2.set_state(blob)
    assert s2.t == 25
    s2.step(35)
    assert np.array_equal(s2.fields(), straight)


def test_determinism():
    g, prob = maxcut_problem(seed=8)
    h0 = W.initial_fields(g.n, 128, seed=8)
    a, sa = run_fields(prob, h0, 128, 50)
    b, sb = run_fields(prob, h0, 128, 50)
    assert np.array_equal(a, b)
    assert np.array_equal(sa.energies()[2], sb.energies()[2])


def test_tuning_restores_the_state(tmp_path, monkeypatch):
    """fem_tune times every shape (twice each) from a device-side backup:
    afterwards the solver continues exactly as one that was never tuned, the
    chosen shape is reported, and it is cached under FEM_TUNE_CACHE."""
    monkeypatch.setenv("FEM_TUNE_CACHE", str(tmp_path / "tune.txt"))
    g, prob = maxcut_problem(n=900, seed=12)
    R = 64
    h0 = W.initial_fields(g.n, R, seed=12)
    ref, _ = run_fields(prob, h0, R, 30, energy_every=1)
    s = fem.Solver(prob, fem.default_params(replicas=R, steps=200, energy_every=1))
    s.set_fields(h0)
    s.step(10)
    tile = s.tune(trial_steps=3, use_cache=False)
    assert tile == s.tile()
    s.step(20)
    assert np.array_equal(s.fields(), ref)
    assert (tmp_path / "tune.txt").read_text().split()[-5:] == [str(v) for v in tile]


@pytest.mark.parametrize("kind", ["maxcut", "maxcut_dense_rows", "maxsat", "bmincut"])
def test_every_tile_shape_gives_identical_fields(kind):
    R = 64
    if kind == "maxcut":
        g, prob = maxcut_problem(n=1500, seed=9)
        h0 = W.initial_fields(g.n, R, seed=9)
        shapes = [(1, 4, 4), (2, 1, 1, 1), (4, 8, 2), (4, 8, 2, 1), (8, 2, 16), (8, 4, 4, 1), (4, 16, 1),
                  (4, 4, 4, 1, 2), (1, 8, 2, 0, 8)]
        kw = {}
    elif kind == "maxcut_dense_rows":
        # mean degree 40: one value per lane takes rows in rounds of sixteen
        # and eight, more values per lane in rounds of four; same sums
        g = W.random_sparse_graph(600, 12000, seed=19, weights="pm1")
        prob = fem.Problem.maxcut(g.n, g.u, g.v, g.w)
        h0 = W.initial_fields(g.n, R, seed=19)
        shapes = [(1, 4, 4), (4, 4, 4), (1, 2, 1, 0, 8), (2, 8, 2, 1), (8, 1, 3)]
        kw = {}
    elif kind == "maxsat":
        cnf = W.random_ksat(1500, 12000, 3, seed=9)
        prob = fem.Problem.maxsat(cnf.n_vars, cnf.clause_off, cnf.lits)
        h0 = W.initial_fields(cnf.n_vars, R, seed=9)
        shapes = [(1, 4, 4), (2, 2, 3, 1), (4, 8, 1), (8, 1, 8, 1), (4, 4, 2, 1, 4)]
        kw = {}
    else:
        g = W.rgg_3d(900, 14.0, seed=9)
        prob = fem.Problem.bmincut(g.n, g.u, g.v, g.w, 4)
        h0 = W.initial_fields(g.n, R, seed=9, q=4)
        shapes = [(4, 4, 4), (4, 1, 1, 1), (4, 8, 3), (4, 2, 16, 1), (4, 4, 2, 0, 16)]
        kw = {"lam": 1.0}
    ref = None
    for sh in shapes:
        h, s = run_fields(prob, h0, R, 30, tile=sh, **kw)
        if ref is None:
            ref = h
        assert np.array_equal(h, ref), sh


def test_replica_independence_bitexact():
    g, prob = maxcut_problem(seed=10)
    h0 = W.initial_fields(g.n, 64, seed=10)
    full, _ = run_fields(prob, h0, 64, 40)
    for r in (0, 17, 63):
        one, _ = run_fields(prob, np.ascontiguousarray(h0[:, r:r + 1]), 1, 40)
        assert np.array_equal(one[:, 0], full[:, r])


def test_batch_equals_standalone():
    """A block-diagonal batch of uneven instances reproduces every instance run
    alone: fields bit for bit, energies and best cuts per instance."""
    R = 32
    graphs = [W.batch_instance(b, n_override=n) for b, n in enumerate([1000, 1373, 2002, 1111, 3000])]
    parts = [fem.Problem.maxcut(g.n, g.u, g.v, g.w) for g in graphs]
    batch = fem.Problem.batch(parts)
    assert batch.n_inst == 5 and batch.n == sum(g.n for g in graphs)
    offs = batch.instance_offsets()
    h0s = [W.initial_fields(g.n, R, seed=1_000_000 + 50_000 + b) for b, g in enumerate(graphs)]
    hb, sb = run_fields(batch, np.concatenate(h0s), R, 60, eval_every=20)
    Ub, Sb, Fb = sb.energies()
    repb, valb, sigb = sb.best()
    for b, (g, p) in enumerate(zip(graphs, parts)):
        hs, ss = run_fields(p, h0s[b], R, 60, eval_every=20)
        assert np.array_equal(hb[offs[b]:offs[b + 1]], hs), b
        U, S, F = ss.energies()
        assert np.array_equal(U[0], Ub[b]) and np.array_equal(S[0], Sb[b])
        rep, val, sig = ss.best()
        assert rep[0] == repb[b] and val[0] == valb[b]
        assert np.array_equal(sig, sigb[offs[b]:offs[b + 1]])
        assert np.array_equal(ss.anytime_best()[0], sb.anytime_best()[b])


def test_anytime_best_tracks_evaluations():
    g, prob = maxcut_problem(seed=12)
    R = 16
    h0 = W.initial_fields(g.n, R, seed=12)
    s = fem.Solver(prob, fem.default_params(replicas=R, steps=100, eval_every=25))
    s.set_fields(h0)
    seen = np.full(R, -np.inf)
    for _ in range(4):
        s.step(25)
        vals, _ = prob.eval_int(s.round())
        seen = np.maximum(seen, vals[0])
        assert np.array_equal(s.anytime_best()[0], seen)


def test_error_states():
    g, prob = maxcut_problem(n=200, seed=13)
    s = fem.Solver(prob, fem.default_params(replicas=4, steps=10))
    with pytest.raises(fem.FemError) as ei:
        s.step(1)
    assert ei.value.status == fem.FEM_E_STATE
    with pytest.raises(fem.FemError) as ei:
        s.energies()
    assert ei.value.status == fem.FEM_E_STATE
    s.set_fields(W.initial_fields(g.n, 4, seed=1))
    with pytest.raises(fem.FemError) as ei:
        s.step(11)
    assert ei.value.status == fem.FEM_E_STATE
    with pytest.raises(fem.FemError) as ei:
        s.last_grad()
    assert ei.value.status == fem.FEM_E_STATE
    with pytest.raises(fem.FemError) as ei:
        s.set_tile(3, 4, 4)
    assert ei.value.status == fem.FEM_E_INVAL
    with pytest.raises(fem.FemError) as ei:
        fem.Solver(prob, fem.default_params(replicas=4, steps=10, beta_min=0.0))
    assert ei.value.status == fem.FEM_E_INVAL
    with pytest.raises(fem.FemError) as ei:
        fem.Solver(prob, fem.default_params(replicas=1 << 30, steps=10))
    assert ei.value.status == fem.FEM_E_NOMEM


def test_nan_fields_reported():
    g, prob = maxcut_problem(n=300, seed=14)
    h = W.initial_fields(g.n, 8, seed=2)
    h[5, 3] = np.nan
    s = fem.Solver(prob, fem.default_params(replicas=8, steps=10))
    s.set_fields(h)
    s.step(1)
    with pytest.raises(fem.FemError) as ei:
        s.energies()
    assert ei.value.status == fem.FEM_E_NUMERIC


def test_device_pointers_from_torch():
    g, prob = maxcut_problem(n=500, seed=15)
    R = 32
    h0 = W.initial_fields(g.n, R, seed=3)
    ref, _ = run_fields(prob, h0, R, 20)
    st = torch.cuda.Stream()
    s = fem.Solver(prob, fem.default_params(replicas=R, steps=200), stream=st)
    s.set_fields(torch.from_numpy(h0).cuda())
    s.step(20)
    out = torch.empty(g.n, R, device="cuda")
    s.fields(out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref)


@pytest.mark.parametrize("kind", ["maxcut", "maxsat", "bmincut", "manip"])
def test_state_layouts_are_bitexact(kind):
    """The interleaved layout of h and the Adam moments changes nothing but
    how they are streamed: fields, gradients, read-out and checkpoints agree
    bit for bit with the separate layout."""
    R = 48
    kw = {}
    if kind in ("maxcut", "manip"):
        g, prob = maxcut_problem(n=900, seed=21)
        h0 = W.initial_fields(g.n, R, seed=21)
        if kind == "manip":
            kw = dict(gradient=fem.GRAD_MANIPULATED, energy_every=0)
    elif kind == "maxsat":
        cnf = W.random_ksat(800, 6000, 3, seed=21)
        prob = fem.Problem.maxsat(cnf.n_vars, cnf.clause_off, cnf.lits)
        h0 = W.initial_fields(cnf.n_vars, R, seed=21)
    else:
        g = W.rgg_3d(700, 12.0, seed=21)
        prob = fem.Problem.bmincut(g.n, g.u, g.v, g.w, 4)
        h0 = W.initial_fields(g.n, R, seed=21, q=4)
        kw = {"lam": 0.7}
    out = []
    for layout in (fem.STATE_SEPARATE, fem.STATE_INTERLEAVED):
        h, s = run_fields(prob, h0, R, 25, keep_grad=1, state_layout=layout, **kw)
        out.append((h, s.last_grad(), s.round(), s.get_state()))
    for a, b in zip(out[0][:3], out[1][:3]):
        assert np.array_equal(a, b)
    assert out[0][3] == out[1][3]
    # a checkpoint written in one layout resumes in the other
    s2 = fem.Solver(prob, fem.default_params(replicas=R, steps=200, state_layout=fem.STATE_INTERLEAVED, **kw))
    s2.set_state(out[0][3])
    s2.step(5)
    s1 = fem.Solver(prob, fem.default_params(replicas=R, steps=200, **kw))
    s1.set_state(out[0][3])
    s1.step(5)
    assert np.array_equal(s1.fields(), s2.fields())
