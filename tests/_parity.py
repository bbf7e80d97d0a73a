"""Comparison helpers for GPU-vs-oracle parity tests.

Tolerances (fixed by the workload description): float32 gradients and
energies within 1e-5 relative of the FP64 oracle; gradients per replica
norm-wise and element-wise (max |dg| <= 1e-5 * max |g_ref|).  Each energy is
judged against its own scale: U against the summed magnitude of the terms it
is formed from (so that +/-1 weights cancelling in U do not make the bar
vacuous or impossible), S against |S|, and F = U - S/beta, a difference of
two large terms, against max(scale of U, |S| / beta).

With a bfloat16 marginal copy the oracle rounds its own FP64 marginals to
bfloat16; the GPU rounds its float32 ones.  The two agree except where a
value lies within float32 error of a rounding midpoint, and there they differ
by one bfloat16 step.  ``bf16_slack`` finds those values from the state and
bounds what they can change; everywhere else the 1e-5 bar holds unchanged.
"""
import numpy as np

import oracle as O

RTOL = 1e-5
# float32 error of a computed marginal, in float32 ulps, within which the
# two sides may round to different bfloat16 neighbours
AMBIG_ULPS = 16


def per_replica(x, R):
    """[n][R] or [n][R][q] -> [R][n*q]"""
    x = np.asarray(x, dtype=np.float64)
    return np.moveaxis(x.reshape(x.shape[0], R, -1), 1, 0).reshape(R, -1)


def grad_errors(g_gpu, g_ref, R, mask=None):
    """Per replica: norm-wise relative error (over the elements where mask is
    true, if given) and max |dg| / max |g_ref|."""
    a, b = per_replica(g_gpu, R), per_replica(g_ref, R)
    nrm = np.linalg.norm(b, axis=1)
    d = a - b
    dn = d if mask is None else np.where(per_replica(mask, R) > 0, d, 0.0)
    rel = np.linalg.norm(dn, axis=1) / np.maximum(nrm, 1e-300)
    mx = np.abs(d).max(axis=1) / np.maximum(np.abs(b).max(axis=1), 1e-300)
    return rel, mx


def assert_grad_close(g_gpu, g_ref, R, rtol=RTOL, what="g", slack=None):
    """1e-5 bar per replica; with slack (absolute, per element, from values
    that may round to different bfloat16 neighbours) the element-wise bound
    becomes rtol * max|g_ref| + slack and the norm-wise one is taken over the
    elements without slack."""
    if slack is None:
        rel, mx = grad_errors(g_gpu, g_ref, R)
        assert rel.max() <= rtol and mx.max() <= rtol, f"{what}: norm rel {rel.max():.3e}, max rel {mx.max():.3e}"
        return rel.max(), mx.max()
    clean = slack == 0
    rel, _ = grad_errors(g_gpu, g_ref, R, mask=clean)
    err = np.abs(np.asarray(g_gpu, np.float64) - g_ref)
    tol = rtol * per_replica_max(g_ref, R) + slack
    bad = err > tol
    assert rel.max() <= rtol and not bad.any(), \
        f"{what}: norm rel (values without slack) {rel.max():.3e}, {int(bad.sum())} values above the bound, " \
        f"worst excess {float((err - tol).max()):.3e}"
    mx = float((np.where(clean, err, 0.0) / np.maximum(per_replica_max(g_ref, R), 1e-300)).max())
    return rel.max(), mx


def energy_errors(U, S, F, Ur, Sr, beta, uscale=None, uslack=0.0):
    """Relative errors of U (against uscale, default |U_ref|, after removing
    uslack), S (against |S_ref|) and F (against max(uscale, |S_ref|/beta))."""
    us = np.abs(Ur) if uscale is None else uscale
    fscale = np.maximum(us, np.abs(Sr) / beta)
    Fr = Ur - Sr / beta
    eu = (np.maximum(np.abs(U - Ur) - uslack, 0.0) / np.maximum(us, 1e-300)).max()
    es = (np.abs(S - Sr) / np.maximum(np.abs(Sr), 1e-300)).max()
    ef = (np.maximum(np.abs(F - Fr) - uslack, 0.0) / np.maximum(fscale, 1e-300)).max()
    return eu, es, ef


def assert_energy_close(U, S, F, Ur, Sr, beta, rtol=RTOL, what="E", uscale=None, uslack=0.0):
    eu, es, ef = energy_errors(U, S, F, Ur, Sr, beta, uscale, uslack)
    assert max(eu, es, ef) <= rtol, f"{what}: U {eu:.3e} S {es:.3e} F {ef:.3e}"
    return eu, es, ef


def per_replica_max(x, R):
    """max |x| per replica, broadcast back to the layout of x."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    m = x.reshape(x.shape[0], R, -1).max(axis=(0, 2))
    shape = (1, R) + (1,) * (x.ndim - 2)
    return m.reshape(shape)


# ---------------------------------------------------------------------------
# Energy scales and bfloat16 slack, from the (float32) state the step starts
# from.  These only size tolerances; the reference values are the oracle's.
# ---------------------------------------------------------------------------
def _softmax(h):
    e = np.exp(h - h.max(axis=-1, keepdims=True))
    return e / e.sum(axis=-1, keepdims=True)


def _sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def _clauses(off, lits):
    """Canonical clauses (distinct variables in first-occurrence order,
    clauses holding x and not-x dropped) as lists of variables."""
    out = []
    for m in range(len(off) - 1):
        seen, taut = {}, False
        for L in lits[off[m]:off[m + 1]]:
            x, pos = abs(int(L)) - 1, L > 0
            if x in seen:
                taut = taut or seen[x] != pos
            else:
                seen[x] = pos
        if not taut:
            out.append(list(seen))
    return out


def _abs_adjacency(run):
    """|W| as a symmetric sparse matrix (cached on the run)."""
    A = getattr(run, "_absW", None)
    if A is None:
        import scipy.sparse as sp

        u, v, w = run._keep
        aw = np.abs(np.asarray(w, dtype=np.float64))
        A = sp.csr_matrix((np.concatenate([aw, aw]), (np.concatenate([u, v]), np.concatenate([v, u]))),
                          shape=(run.n, run.n))
        run._absW = A
    return A


def _spmm(A, x):
    """A @ x over the first axis of x (any trailing shape)."""
    return np.asarray(A @ x.reshape(x.shape[0], -1)).reshape(x.shape)


def u_scale(run, h, t):
    """Summed magnitude of the terms U is formed from, per replica (None for
    Max-k-SAT, whose U is a sum of non-negative terms: |U| itself)."""
    h = np.asarray(h, dtype=np.float64)
    if run.kind == O.KIND_MAXCUT:
        A = _abs_adjacency(run)
        am = np.abs(np.tanh(0.5 * h))
        # sum over edges |W| (1 + |m_u m_v|)
        return 0.5 * A.sum() + 0.5 * np.sum(am * _spmm(A, am), axis=0)
    if run.kind == O.KIND_BMINCUT:
        p = run.p
        A = _abs_adjacency(run)
        P = _softmax(h)
        V = np.ones(h.shape[0]) if run.node_w is None else run.node_w
        C = np.einsum("i,irs->rs", V, P)
        lam = O.lam(p.lam_ramp, p.lam, p.T, t)
        # ordered pairs: sum |W| (1 + P_i . P_j)
        cut = A.sum() + np.sum(P * _spmm(A, P), axis=(0, 2))
        bal = np.sum(C * C, axis=1) + np.einsum("i,irs->r", V * V, P * P)
        return cut + abs(lam) * bal
    return None


def _ambiguous(x):
    """(ambiguous, bfloat16 spacing) of stored values x: ambiguous where x
    lies within AMBIG_ULPS float32 ulps of a bfloat16 rounding midpoint."""
    ax = np.abs(x)
    _, e = np.frexp(ax)
    step = np.ldexp(1.0, np.maximum(e - 8, -133))
    r = ax / step
    dist = np.abs(r - np.floor(r) - 0.5) * step
    f32ulp = np.ldexp(1.0, np.maximum(e - 24, -149))
    return (dist <= AMBIG_ULPS * f32ulp) & (ax > 0), step


def bf16_slack(run, h, t):
    """(gradient slack [layout of h], U slack [R]): the largest change that
    the stored values which may round differently on the two sides can make."""
    h = np.asarray(h, dtype=np.float64)
    if run.kind == O.KIND_MAXCUT:
        m = np.tanh(0.5 * h)
        amb, step = _ambiguous(m)
        dphi = _spmm(_abs_adjacency(run), np.where(amb, step, 0.0))
        p = _sigmoid(h)
        return p * (1 - p) * 2.0 * dphi, 0.5 * np.sum(np.abs(m) * dphi, axis=0)
    if run.kind == O.KIND_BMINCUT:
        P = _softmax(h)
        amb, step = _ambiguous(P)
        dphi = _spmm(_abs_adjacency(run), np.where(amb, step, 0.0))
        dA = 2.0 * dphi
        gs = P * (dA + np.sum(P * dA, axis=2, keepdims=True))
        return gs, np.sum(P * dphi, axis=(0, 2))
    off, lits = run._keep
    small = _sigmoid(-np.abs(h))
    amb, step = _ambiguous(small)
    du = np.where(amb, step, 0.0)
    dd = np.zeros_like(h)
    dU = np.zeros(h.shape[1])
    for cl in _clauses(off, lits):
        tot = du[cl].sum(axis=0)
        for x in cl:
            dd[x] += tot - du[x]
        dU += tot - du[cl[0]]
    p = _sigmoid(h)
    return p * (1 - p) * dd, dU


# ---------------------------------------------------------------------------
# Lockstep parity along the oracle's trajectory.
#
# Free-running FP32 and FP64 trajectories separate: Adam's first step is
# -lr * g / (|g| + eps), a sign function wherever |g| is tiny, and the anneal
# amplifies any difference after the ordering transition.  So each step t is
# checked from the oracle's own state (h, m1, m2, t), rounded to float32 and
# loaded into the GPU solver: data flows from the oracle to the GPU only.  The
# reference values of step t are the oracle's, evaluated at that float32
# state (the state the GPU holds), so the check judges the GPU's arithmetic
# rather than the rounding of its inputs.  The GPU's gradient and energies at
# step t must match them to RTOL; its h(t+1) must lie within the deviation that
# Adam's update shows when the gradient moves within the gradient tolerance
# (evaluated in FP64 on a grid of the interval), plus RTOL * max |h(t+1)|.
# ---------------------------------------------------------------------------
def oracle_trajectory(run, n_steps):
    states, gs, Us, Ss = [], [], [], []
    for _ in range(n_steps):
        states.append((run.h.copy(), run.m1.copy(), run.m2.copy()))
        g, U, S = run.step(1, record=True)
        gs.append(g[0]); Us.append(U[0]); Ss.append(S[0])
    states.append((run.h.copy(), run.m1.copy(), run.m2.copy()))
    return states, gs, Us, Ss


def adam_deviation(h, m1, m2, g, t, p, dg, npts=9):
    """max_{|e| <= dg} |U(h, m1, m2, g + e) - U(h, m1, m2, g)| (FP64), U the
    optimiser update (Adam, or RMSprop / SGD when p.opt says so)."""
    n = t + 1
    bc1 = 1 - p.b1 ** n
    bc2s = np.sqrt(1 - p.b2 ** n)
    opt = getattr(p, "opt", 0)

    def upd(gg):
        gg = gg + p.wd * h
        if opt == 1:
            b = p.rms_alpha * m2 + (1 - p.rms_alpha) * gg * gg
            d = np.sqrt(b) + p.eps
            if p.momentum > 0:
                return h - p.lr * (p.momentum * m1 + gg / d)
            return h - p.lr * gg / d
        if opt == 2:
            if p.momentum != 0:
                gg = gg if t == 0 else p.momentum * m1 + (1 - p.dampening) * gg
            return h - p.lr * gg
        a = p.b1 * m1 + (1 - p.b1) * gg
        b = p.b2 * m2 + (1 - p.b2) * gg * gg
        return h - (p.lr / bc1) * a / (np.sqrt(b) / bc2s + p.eps)

    base = upd(g)
    dev = np.zeros_like(g)
    for x in np.linspace(-1.0, 1.0, npts):
        dev = np.maximum(dev, np.abs(upd(g + x * dg) - base))
    return dev


def lockstep(solver, run, params, n_steps, R, tag, betas, energies=True, rtol=RTOL):
    """Run the oracle n_steps, then replay every step on the GPU from the
    oracle's state; returns the worst relative errors."""
    states, _, _, _ = oracle_trajectory(run, n_steps)
    worst = dict(g=0.0, E=0.0, h=0.0)
    n_slack = 0
    for t in range(n_steps):
        h, m1, m2 = (x.astype(np.float32).astype(np.float64) for x in states[t])
        gref, Uref, Sref = run.eval_at(h, t)
        href = run.adam_from(h, m1, m2, gref, t)
        solver.set_adam_state(h, m1, m2, t)
        solver.step(1)
        gslack, uslack = bf16_slack(run, h, t) if getattr(params, "mdt", 0) else (None, 0.0)
        if gslack is not None:
            n_slack += int(np.count_nonzero(gslack))
        a, b = assert_grad_close(solver.last_grad(), gref, R, rtol=rtol, what=f"{tag} g step {t}", slack=gslack)
        worst["g"] = max(worst["g"], a, b)
        if energies:
            U, S, F = solver.energies()
            e = assert_energy_close(U[0], S[0], F[0], Uref, Sref, betas[t], rtol=rtol,
                                    what=f"{tag} energies step {t}", uscale=u_scale(run, h, t), uslack=uslack)
            worst["E"] = max(worst["E"], *e)
        hn = solver.fields().astype(np.float64)
        dg = rtol * per_replica_max(gref, R) + (0.0 if gslack is None else gslack)
        tol = adam_deviation(h, m1, m2, gref, t, params, dg) + rtol * per_replica_max(href, R)
        err = np.abs(hn - href)
        bad = err > tol
        assert not bad.any(), f"{tag} h({t + 1}): {int(bad.sum())} values outside the propagated tolerance, " \
                              f"worst excess {float((err - tol).max()):.3e}"
        worst["h"] = max(worst["h"], float((err / np.maximum(per_replica_max(href, R), 1e-300)).max()))
    extra = f", values with bf16 rounding slack {n_slack} of {n_steps * h.size}" if getattr(params, "mdt", 0) else ""
    print(f"[{tag}] lockstep {n_steps} steps: worst rel error grad {worst['g']:.2e}, energies {worst['E']:.2e}, "
          f"h {worst['h']:.2e}{extra}", flush=True)
    return worst


def free_running_drift(grads, gref, R):
    """Per-step norm-wise relative gradient error of a free-running pair."""
    return [float(grad_errors(grads[t], gref[t], R)[0].max()) for t in range(len(grads))]


def lockstep_batch(solver, runs, offsets, params, n_steps, R, tag, betas, energies=True, rtol=RTOL):
    """Lockstep of a block-diagonal batch against one oracle run per
    instance: at every step the instances' oracle states are concatenated
    into the batch solver, one batched step runs, and each instance's
    gradient, energies and h(t+1) are judged against its own oracle run as in
    ``lockstep``.  With eval_every = 1 the anytime best of every (instance,
    replica) must then equal the best cut of the oracle's own read-outs,
    wherever no field of the replica was within the h tolerance of zero (the
    read-out's sign would be undecided there; such replicas are counted)."""
    B = len(runs)
    trajs = [oracle_trajectory(run, n_steps)[0] for run in runs]
    worst = dict(g=0.0, E=0.0, h=0.0)
    maximise = runs[0].kind == O.KIND_MAXCUT
    ref_best = np.full((B, R), -np.inf if maximise else np.inf)
    undecided = np.zeros((B, R), dtype=bool)
    for t in range(n_steps):
        st = [[x.astype(np.float32).astype(np.float64) for x in trajs[b][t]] for b in range(B)]
        solver.set_adam_state(*(np.concatenate([st[b][k] for b in range(B)]) for k in range(3)), t)
        solver.step(1)
        g = solver.last_grad().astype(np.float64)
        hn = solver.fields().astype(np.float64)
        if energies:
            U, S, F = solver.energies()
        for b, run in enumerate(runs):
            lo, hi = offsets[b], offsets[b + 1]
            h, m1, m2 = st[b]
            gref, Uref, Sref = run.eval_at(h, t)
            href = run.adam_from(h, m1, m2, gref, t)
            gslack, uslack = bf16_slack(run, h, t) if getattr(params, "mdt", 0) else (None, 0.0)
            a, c = assert_grad_close(g[lo:hi], gref, R, rtol=rtol, what=f"{tag} instance {b} g step {t}",
                                     slack=gslack)
            worst["g"] = max(worst["g"], a, c)
            if energies:
                e = assert_energy_close(U[b], S[b], F[b], Uref, Sref, betas[t], rtol=rtol,
                                        what=f"{tag} instance {b} energies step {t}", uscale=u_scale(run, h, t),
                                        uslack=uslack)
                worst["E"] = max(worst["E"], *e)
            dg = rtol * per_replica_max(gref, R) + (0.0 if gslack is None else gslack)
            tol = adam_deviation(h, m1, m2, gref, t, params, dg) + rtol * per_replica_max(href, R)
            err = np.abs(hn[lo:hi] - href)
            assert not (err > tol).any(), f"{tag} instance {b} h({t + 1}) outside the propagated tolerance"
            worst["h"] = max(worst["h"], float((err / np.maximum(per_replica_max(href, R), 1e-300)).max()))
            # the oracle's read-out of its own h(t+1)
            h1 = trajs[b][t + 1][0]
            if run.kind != O.KIND_BMINCUT:
                undecided[b] |= np.any(np.abs(h1) <= tol, axis=0)
            else:
                srt = np.sort(h1, axis=2)
                undecided[b] |= np.any(srt[:, :, -1] - srt[:, :, -2] <= 2 * tol.max(axis=2), axis=0)
            val = instance_value(run, O.round_(h1, run.q if run.kind == O.KIND_BMINCUT else 1))
            ref_best[b] = np.maximum(ref_best[b], val) if maximise else np.minimum(ref_best[b], val)
    print(f"[{tag}] batch lockstep {n_steps} steps over {B} instances: worst rel error grad {worst['g']:.2e}, "
          f"energies {worst['E']:.2e}, h {worst['h']:.2e}; replicas with an undecided read-out "
          f"{int(undecided.sum())} of {B * R}", flush=True)
    return worst, ref_best, undecided


def instance_value(run, sigma):
    """The value the read-out keeps for configurations sigma [R][n] of one
    instance: the cut (MaxCut, higher is better), the number of unsatisfied
    clauses (Max-k-SAT) or the integer bMinCut energy
    2 cut + lambda (sum_s W_s^2 - sum_i V_i^2) with the solver's lambda (lower
    is better)."""
    if run.kind == O.KIND_MAXCUT:
        u, v, w = run._keep
        return O.cut(run.n, u, v, w, sigma)
    if run.kind == O.KIND_MAXSAT:
        off, lits = run._keep
        return O.unsat(run.n, off, lits, sigma).astype(np.float64)
    u, v, w = run._keep
    V = None if run.node_w is None else run.node_w.astype(np.int32)
    sz = O.group_sizes(run.n, run.q, sigma, node_w=V).astype(np.float64)
    v2 = float(run.n) if V is None else float(np.sum(V.astype(np.float64) ** 2))
    return 2 * O.cut(run.n, u, v, w, sigma) + run.p.lam * (np.sum(sz * sz, axis=1) - v2)
