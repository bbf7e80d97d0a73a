"""GPU parity of the Max-k-SAT (clause-product gradient) hot path against the
FP64 oracle, through the C ABI.  Seeded inputs only; step parity is lockstep
along the oracle's trajectory (oracle -> GPU only)."""
import numpy as np
import pytest

import oracle as O
from paper_2412_09285_amd import fem
from paper_2412_09285_amd import workloads as W
from _parity import assert_energy_close, assert_grad_close, grad_errors, lockstep

pytestmark = pytest.mark.gpu


def mixed_cnf(n, M, seed):
    """Clauses of 1..4 literals, with repeated literals and tautologies."""
    rng = np.random.default_rng(seed)
    clauses = []
    for m in range(M):
        k = int(rng.integers(1, 5))
        vs = rng.choice(n, size=k, replace=False)
        c = [int(x + 1) if rng.random() < 0.5 else -int(x + 1) for x in vs]
        if m % 17 == 0:
            c.append(c[0])           # repeated literal
        if m % 29 == 0:
            c.append(-c[0])          # tautology
        clauses.append(c)
    off = np.cumsum([0] + [len(c) for c in clauses]).astype(np.int64)
    lits = np.array([x for c in clauses for x in c], dtype=np.int32)
    return W.CNF(n, off, lits)


def free_run(cnf, R, T, n_steps, seed, dtype=fem.F32, tile=None):
    h0 = W.initial_fields(cnf.n_vars, R, seed)
    prob = fem.Problem.maxsat(cnf.n_vars, cnf.clause_off, cnf.lits)
    s = fem.Solver(prob, fem.default_params(replicas=R, steps=T, keep_grad=1, record_energies=1,
                                            marginal_dtype=dtype))
    if tile is not None:
        s.set_tile(*tile)
    s.set_fields(h0)
    grads = []
    for _ in range(n_steps):
        s.step(1)
        grads.append(s.last_grad())
    U, S, F = s.energy_history(0, n_steps)
    run = O.maxsat_run(cnf, O.Params(R=R, T=T), h0)
    gh, Uh, Sh = run.step(n_steps, record=True)
    betas = np.array([O.beta(0, 0.01, 5.0, T, t) for t in range(n_steps)])
    return dict(grads=np.array(grads), U=U[:, 0], S=S[:, 0], F=F[:, 0], h=s.fields(), gref=gh, Uref=Uh,
                Sref=Sh, href=run.h, betas=betas)


def lockstep_sat(cnf, R, T, n_steps, seed, tile=None, tag="", dtype=fem.F32):
    h0 = W.initial_fields(cnf.n_vars, R, seed)
    prob = fem.Problem.maxsat(cnf.n_vars, cnf.clause_off, cnf.lits)
    s = fem.Solver(prob, fem.default_params(replicas=R, steps=T, keep_grad=1, marginal_dtype=dtype))
    if tile is not None:
        s.set_tile(*tile)
    P = O.Params(R=R, T=T, mdt=int(dtype == fem.BF16))
    run = O.maxsat_run(cnf, P, h0)
    betas = [O.beta(0, P.beta_min, P.beta_max, T, t) for t in range(n_steps)]
    return lockstep(s, run, P, n_steps, R, tag, betas)


def test_random_3sat_first_100_steps():
    """The Max-3-SAT recipe (ratio 8, distinct variables, fair signs) at
    N = 2,000, R = 64: the first 100 steps."""
    lockstep_sat(W.random_ksat(2000, 16000, 3, seed=4), R=64, T=2000, n_steps=100, seed=104, tag="3sat2000")


@pytest.mark.parametrize("R", [1, 16, 24])
def test_mixed_lengths_repeats_tautologies(R):
    lockstep_sat(mixed_cnf(300, 1500, seed=R), R=R, T=300, n_steps=40, seed=R + 1, tag=f"mixed_R{R}")


@pytest.mark.parametrize("vec,waves,rows,lanes", [(1, 2, 1, 0), (2, 4, 5, 0), (4, 8, 2, 0), (4, 4, 3, 4),
                                                (2, 2, 2, 8)])
def test_tile_shapes(vec, waves, rows, lanes):
    lockstep_sat(W.random_ksat(1000, 8000, 3, seed=8), R=64, T=100, n_steps=10, seed=5,
                 tile=(vec, waves, rows, 0, lanes), tag=f"tile{vec}x{waves}x{rows}L{lanes}")


def test_unsat_count_bitexact():
    rng = np.random.default_rng(2)
    for cnf in (W.random_ksat(3000, 24000, 3, seed=9), mixed_cnf(400, 3000, seed=3)):
        prob = fem.Problem.maxsat(cnf.n_vars, cnf.clause_off, cnf.lits)
        sigma = rng.integers(0, 2, size=(33, cnf.n_vars)).astype(np.int32)
        vals, _ = prob.eval_int(sigma)
        ref = O.unsat(cnf.n_vars, cnf.clause_off, cnf.lits, sigma)
        assert np.array_equal(vals[0], ref)


def test_paper_example_cnf():
    """The worked CNF of the Max-k-SAT section: every assignment is counted as
    the definition says, and the optimum is 0."""
    clauses = [[1, -2, -2], [-1, 4], [2, -3, -4]]
    off = np.cumsum([0] + [len(c) for c in clauses]).astype(np.int64)
    lits = np.array([x for c in clauses for x in c], dtype=np.int32)
    prob = fem.Problem.maxsat(4, off, lits)
    import itertools

    allsig = np.array(list(itertools.product((0, 1), repeat=4)), dtype=np.int32)
    vals, _ = prob.eval_int(allsig)
    assert np.array_equal(vals[0], O.unsat(4, off, lits, allsig))
    assert vals.min() == 0


def test_random_3sat_bf16_first_100_steps():
    """BF16 copy of min(P, 1 - P): the first 100 steps against the oracle
    with the same bfloat16 copy, 1e-5 except where the two sides may round a
    stored value to different bfloat16 neighbours."""
    lockstep_sat(W.random_ksat(2000, 16000, 3, seed=4), R=64, T=2000, n_steps=100, seed=104, dtype=fem.BF16,
                 tag="3sat2000 bf16")


def test_mixed_lengths_bf16():
    lockstep_sat(mixed_cnf(300, 1500, seed=5), R=16, T=300, n_steps=40, seed=6, dtype=fem.BF16, tag="mixed bf16")


def test_config4_full_size_two_steps():
    """N = 100,000 variables, M = 800,000 3-clauses, R = 64 in the tuned launch
    shape: the first two steps lockstep with the oracle on all replicas."""
    cnf = W.config_cnf(4)
    R, T = 64, 2000
    h0 = W.initial_fields(cnf.n_vars, R, seed=104)
    prob = fem.Problem.maxsat(cnf.n_vars, cnf.clause_off, cnf.lits)
    s = fem.Solver(prob, fem.default_params(replicas=R, steps=T, keep_grad=1))
    s.set_fields(h0)
    tile = s.tune(trial_steps=3, use_cache=True)
    P = O.Params(R=R, T=T)
    run = O.maxsat_run(cnf, P, h0)
    lockstep(s, run, P, 2, R, f"C4 full, tile {tile}", [O.beta(0, 0.01, 5.0, T, t) for t in range(2)])
