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
