"""Comparison helpers for GPU-vs-oracle parity tests.

Tolerances (fixed by the workload description): float32 gradients and
energies within 1e-5 relative of the FP64 oracle, norm-wise per replica; for
gradients also max |dg| <= 1e-5 * max |g_ref| per replica.  Energies are
compared with the scale max(|U|, |S| / beta), so that F = U - S/beta, a
difference of two large terms, is judged against the terms that form it.
"""
import numpy as np

RTOL = 1e-5


def per_replica(x, R):
    """[n][R] or [n][R][q] -> [R][n*q]"""
    x = np.asarray(x, dtype=np.float64)
    return np.moveaxis(x.reshape(x.shape[0], R, -1), 1, 0).reshape(R, -1)


def grad_errors(g_gpu, g_ref, R):
    a, b = per_replica(g_gpu, R), per_replica(g_ref, R)
    nrm = np.linalg.norm(b, axis=1)
    rel = np.linalg.norm(a - b, axis=1) / np.maximum(nrm, 1e-300)
    mx = np.abs(a - b).max(axis=1) / np.maximum(np.abs(b).max(axis=1), 1e-300)
    return rel, mx


def assert_grad_close(g_gpu, g_ref, R, rtol=RTOL, what="g"):
    rel, mx = grad_errors(g_gpu, g_ref, R)
    assert rel.max() <= rtol and mx.max() <= rtol, f"{what}: norm rel {rel.max():.3e}, max rel {mx.max():.3e}"
    return rel.max(), mx.max()


def energy_errors(U, S, F, Ur, Sr, beta):
    scale = np.maximum(np.abs(Ur), np.abs(Sr) / beta)
    Fr = Ur - Sr / beta
    return (np.abs(U - Ur) / scale).max(), (np.abs(S - Sr) / np.maximum(np.abs(Sr), 1e-300)).max(), \
        (np.abs(F - Fr) / scale).max()


def assert_energy_close(U, S, F, Ur, Sr, beta, rtol=RTOL, what="E"):
    eu, es, ef = energy_errors(U, S, F, Ur, Sr, beta)
    assert max(eu, es, ef) <= rtol, f"{what}: U {eu:.3e} S {es:.3e} F {ef:.3e}"
    return eu, es, ef


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


def per_replica_max(x, R):
    """max |x| per replica, broadcast back to the layout of x."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    m = x.reshape(x.shape[0], R, -1).max(axis=(0, 2))
    shape = (1, R) + (1,) * (x.ndim - 2)
    return m.reshape(shape)


def lockstep(solver, run, params, n_steps, R, tag, betas, energies=True, rtol=RTOL):
    """Run the oracle n_steps, then replay every step on the GPU from the
    oracle's state; returns the worst relative errors."""
    states, _, _, _ = oracle_trajectory(run, n_steps)
    worst = dict(g=0.0, E=0.0, h=0.0)
    for t in range(n_steps):
        h, m1, m2 = (x.astype(np.float32).astype(np.float64) for x in states[t])
        gref, Uref, Sref = run.eval_at(h, t)
        href = run.adam_from(h, m1, m2, gref, t)
        solver.set_adam_state(h, m1, m2, t)
        solver.step(1)
        a, b = assert_grad_close(solver.last_grad(), gref, R, rtol=rtol, what=f"{tag} g step {t}")
        worst["g"] = max(worst["g"], a, b)
        if energies:
            U, S, F = solver.energies()
            e = assert_energy_close(U[0], S[0], F[0], Uref, Sref, betas[t], rtol=rtol,
                                    what=f"{tag} energies step {t}")
            worst["E"] = max(worst["E"], *e)
        hn = solver.fields().astype(np.float64)
        dg = rtol * per_replica_max(gref, R)
        tol = adam_deviation(h, m1, m2, gref, t, params, dg) + rtol * per_replica_max(href, R)
        err = np.abs(hn - href)
        bad = err > tol
        assert not bad.any(), f"{tag} h({t + 1}): {int(bad.sum())} values outside the propagated tolerance, " \
                              f"worst excess {float((err - tol).max()):.3e}"
        worst["h"] = max(worst["h"], float((err / np.maximum(per_replica_max(href, R), 1e-300)).max()))
    print(f"[{tag}] lockstep {n_steps} steps: worst rel error grad {worst['g']:.2e}, energies {worst['E']:.2e}, "
          f"h {worst['h']:.2e}", flush=True)
    return worst


def free_running_drift(grads, gref, R):
    """Per-step norm-wise relative gradient error of a free-running pair."""
    return [float(grad_errors(grads[t], gref[t], R)[0].max()) for t in range(len(grads))]
