"""FP64 CPU oracle of the Free-Energy Machine step (arXiv 2412.09285).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the product path
(``paper_2412_09285_amd``) never does.  The arithmetic lives in the plain C
file ``fem_oracle.c`` (double precision, single thread, loops in the paper's
order); this module only marshals NumPy arrays to it.

Pinned by ``tests/test_oracle_pins.py``: brute-force expectations over all
configurations, central finite differences of F, closed forms at special
points, the mean-field fixed point, schedule endpoints, Adam against
``torch.optim.Adam`` in float64, brute-force optima and closed-form optimum
families.  The MPNN reference (``oracle.mpnn``) is pinned by finite
differences of its own loss; its training quality is parity unpinned.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fem_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_fem_oracle.so")
_lib = None

KIND_MAXCUT, KIND_BMINCUT, KIND_MAXSAT = 0, 1, 2
SCHED_LINEAR, SCHED_EXP, SCHED_INVPROP = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math) into ``_fem_oracle.so``."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Problem(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("n", C.c_int32), ("q", C.c_int32), ("R", C.c_int32),
        ("T", C.c_int32), ("sched", C.c_int32), ("lam_ramp", C.c_int32),
        ("ne", C.c_int64),
        ("eu", C.c_void_p), ("ev", C.c_void_p), ("w", C.c_void_p),
        ("off", C.c_void_p), ("lits", C.c_void_p),
        ("beta_min", C.c_double), ("beta_max", C.c_double), ("lam", C.c_double),
        ("lr", C.c_double), ("b1", C.c_double), ("b2", C.c_double),
        ("eps", C.c_double), ("wd", C.c_double),
        ("opt", C.c_int32), ("momentum", C.c_double), ("rms_alpha", C.c_double), ("dampening", C.c_double),
        ("manip", C.c_int32), ("gamma", C.c_double), ("nw", C.c_void_p), ("mdt", C.c_int32),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        L.orc_beta.restype = C.c_double
        L.orc_beta.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_int32]
        L.orc_lambda.restype = C.c_double
        L.orc_lambda.argtypes = [C.c_int32, C.c_double, C.c_int32, C.c_int32]
        L.orc_maxcut_grad.restype = C.c_int
        L.orc_round_bf16.restype = C.c_double
        L.orc_round_bf16.argtypes = [C.c_double]
        L.orc_maxcut_grad.argtypes = [C.c_int32, C.c_int64, P, P, P, C.c_int32, P, C.c_double, C.c_int32, P, P, P]
        L.orc_bmincut_grad.restype = C.c_int
        L.orc_bmincut_grad.argtypes = [C.c_int32, C.c_int64, P, P, P, P, C.c_int32, C.c_double,
                                       C.c_int32, P, C.c_double, C.c_int32, P, P, P]
        L.orc_maxsat_grad.restype = C.c_int
        L.orc_maxsat_grad.argtypes = [C.c_int32, C.c_int64, P, P, C.c_int32, P, C.c_double, C.c_int32, P, P, P]
        L.orc_maxcut_grad_manip.restype = C.c_int
        L.orc_maxcut_grad_manip.argtypes = [C.c_int32, C.c_int64, P, P, P, C.c_int32, P, C.c_double,
                                            C.c_double, P]
        L.orc_bmincut_grad_manip.restype = C.c_int
        L.orc_bmincut_grad_manip.argtypes = [C.c_int32, C.c_int64, P, P, P, P, C.c_int32, C.c_double,
                                             C.c_int32, P, C.c_double, C.c_double, P]
        L.orc_maxsat_grad_manip.restype = C.c_int
        L.orc_maxsat_grad_manip.argtypes = [C.c_int32, C.c_int64, P, P, C.c_int32, P, C.c_double,
                                            C.c_double, P]
        L.orc_adam.restype = None
        L.orc_adam.argtypes = [C.c_int64, P, P, P, P, C.c_double, C.c_double, C.c_double,
                               C.c_double, C.c_double, C.c_int64]
        L.orc_rmsprop.restype = None
        L.orc_rmsprop.argtypes = [C.c_int64, P, P, P, P, C.c_double, C.c_double, C.c_double, C.c_double,
                                  C.c_double]
        L.orc_sgd.restype = None
        L.orc_sgd.argtypes = [C.c_int64, P, P, P, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int64]
        L.orc_round.restype = None
        L.orc_round.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P]
        L.orc_cut.restype = None
        L.orc_cut.argtypes = [C.c_int32, C.c_int64, P, P, P, C.c_int32, P, P]
        L.orc_group_sizes.restype = None
        L.orc_group_sizes.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P, P]
        L.orc_unsat.restype = None
        L.orc_unsat.argtypes = [C.c_int32, C.c_int64, P, P, C.c_int32, P, P]
        L.orc_run.restype = C.c_int
        L.orc_run.argtypes = [C.POINTER(_Problem), C.c_int32, C.c_int32, P, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


# --------------------------------------------------------------------------
# schedules
# --------------------------------------------------------------------------
def beta(sched: int, bmin: float, bmax: float, T: int, t: int) -> float:
    return lib().orc_beta(sched, bmin, bmax, T, t)


def lam(ramp: int, lam_max: float, T: int, t: int) -> float:
    return lib().orc_lambda(int(ramp), lam_max, T, t)


# --------------------------------------------------------------------------
# per-step gradient and energies (one call = one evaluation at fixed h, beta)
# --------------------------------------------------------------------------
def round_bf16(x: float) -> float:
    """The nearest bfloat16 value of x (ties to even)."""
    return lib().orc_round_bf16(float(x))


def maxcut_grad(n, u, v, w, h, beta_, want_grad=True, mdt=0):
    """h: [n][R] float64; mdt = 1: neighbours read a bfloat16 copy of m.
    Returns (g [n][R] or None, U [R], S [R])."""
    h = _f64(h)
    R = h.shape[1]
    u, v, w = _i32(u), _i32(v), _f64(w)
    g = np.zeros_like(h) if want_grad else None
    U = np.zeros(R)
    S = np.zeros(R)
    rc = lib().orc_maxcut_grad(n, u.shape[0], _p(u), _p(v), _p(w), R, _p(h), beta_, int(mdt), _p(g), _p(U), _p(S))
    if rc:
        raise MemoryError(rc)
    return g, U, S


def bmincut_grad(n, u, v, w, q, lam_, h, beta_, want_grad=True, node_w=None, mdt=0):
    """h: [n][R][q] float64; node_w: node weights V (None: all 1); mdt = 1:
    neighbours read a bfloat16 copy of P."""
    h = _f64(h)
    R = h.shape[1]
    u, v, w = _i32(u), _i32(v), _f64(w)
    V = None if node_w is None else _f64(node_w)
    g = np.zeros_like(h) if want_grad else None
    U = np.zeros(R)
    S = np.zeros(R)
    rc = lib().orc_bmincut_grad(n, u.shape[0], _p(u), _p(v), _p(w), _p(V), q, lam_, R, _p(h), beta_, int(mdt),
                                _p(g), _p(U), _p(S))
    if rc:
        raise MemoryError(rc)
    return g, U, S


def maxsat_grad(n, off, lits, h, beta_, want_grad=True, mdt=0):
    """mdt = 1: the other literals of a clause are read from a bfloat16 copy
    of min(P, 1 - P)."""
    h = _f64(h)
    R = h.shape[1]
    off, lits = _i64(off), _i32(lits)
    g = np.zeros_like(h) if want_grad else None
    U = np.zeros(R)
    S = np.zeros(R)
    rc = lib().orc_maxsat_grad(n, off.shape[0] - 1, _p(off), _p(lits), R, _p(h), beta_, int(mdt), _p(g), _p(U),
                               _p(S))
    if rc:
        raise MemoryError(rc)
    return g, U, S


def maxcut_grad_manip(n, u, v, w, h, beta_, gamma=1.0):
    """Manipulated MaxCut gradient (one-hot neighbours, 1/sum|W| normalisation);
    h: [n][R] float64.  Returns g [n][R]."""
    h = _f64(h)
    u, v, w = _i32(u), _i32(v), _f64(w)
    g = np.zeros_like(h)
    rc = lib().orc_maxcut_grad_manip(n, u.shape[0], _p(u), _p(v), _p(w), h.shape[1], _p(h), beta_, gamma, _p(g))
    if rc:
        raise MemoryError(rc)
    return g


def bmincut_grad_manip(n, u, v, w, q, lam_, h, beta_, gamma=1.0, node_w=None):
    """Manipulated bMinCut gradient; h: [n][R][q] float64.  Returns g."""
    h = _f64(h)
    u, v, w = _i32(u), _i32(v), _f64(w)
    V = None if node_w is None else _f64(node_w)
    g = np.zeros_like(h)
    rc = lib().orc_bmincut_grad_manip(n, u.shape[0], _p(u), _p(v), _p(w), _p(V), q, lam_, h.shape[1], _p(h), beta_,
                                      gamma, _p(g))
    if rc:
        raise MemoryError(rc)
    return g


def maxsat_grad_manip(n, off, lits, h, beta_, gamma=1.0):
    h = _f64(h)
    off, lits = _i64(off), _i32(lits)
    g = np.zeros_like(h)
    rc = lib().orc_maxsat_grad_manip(n, off.shape[0] - 1, _p(off), _p(lits), h.shape[1], _p(h), beta_, gamma,
                                     _p(g))
    if rc:
        raise MemoryError(rc)
    return g


def rmsprop(g, h, m1, m2, lr, alpha, eps, wd, momentum):
    """In-place RMSprop (torch semantics, not centred) on float64 arrays."""
    for a in (h, m1, m2):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    lib().orc_rmsprop(h.size, _p(g), _p(h), _p(m1), _p(m2), lr, alpha, eps, wd, momentum)


def sgd(g, h, m1, lr, wd, momentum, dampening, n_step):
    """In-place SGD with momentum (torch semantics) on float64 arrays."""
    for a in (h, m1):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    lib().orc_sgd(h.size, _p(g), _p(h), _p(m1), lr, wd, momentum, dampening, int(n_step))


def adam(g, h, m1, m2, lr, b1, b2, eps, wd, n_step):
    """In-place Adam on float64 arrays h, m1, m2 (all contiguous)."""
    for a in (h, m1, m2):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    lib().orc_adam(h.size, _p(g), _p(h), _p(m1), _p(m2), lr, b1, b2, eps, wd, int(n_step))


# --------------------------------------------------------------------------
# read-out and integer evaluation
# --------------------------------------------------------------------------
def round_(h, q: int = 1):
    """sigma [R][n] int32 from fields h ([n][R] if q == 1 else [n][R][q])."""
    h = _f64(h)
    n, R = h.shape[0], h.shape[1]
    sigma = np.zeros((R, n), dtype=np.int32)
    lib().orc_round(n, R, q, _p(h), _p(sigma))
    return sigma


def cut(n, u, v, w, sigma):
    sigma = _i32(sigma)
    R = sigma.shape[0]
    u, v, w = _i32(u), _i32(v), _f64(w)
    out = np.zeros(R)
    lib().orc_cut(n, u.shape[0], _p(u), _p(v), _p(w), R, _p(sigma), _p(out))
    return out


def group_sizes(n, q, sigma, node_w=None):
    """Per replica and state, the summed node weight (the node count when
    node_w is None) of the nodes in that state."""
    sigma = _i32(sigma)
    R = sigma.shape[0]
    V = None if node_w is None else _i32(node_w)
    out = np.zeros((R, q), dtype=np.int64)
    lib().orc_group_sizes(n, q, R, _p(sigma), _p(V), _p(out))
    return out


def unsat(n, off, lits, sigma):
    sigma = _i32(sigma)
    R = sigma.shape[0]
    off, lits = _i64(off), _i32(lits)
    out = np.zeros(R, dtype=np.int64)
    lib().orc_unsat(n, off.shape[0] - 1, _p(off), _p(lits), R, _p(sigma), _p(out))
    return out


# --------------------------------------------------------------------------
# the annealing loop
# --------------------------------------------------------------------------
@dataclass
class Params:
    R: int
    T: int
    beta_min: float = 0.01
    beta_max: float = 5.0
    sched: int = SCHED_LINEAR
    lr: float = 0.1
    b1: float = 0.9
    b2: float = 0.999
    eps: float = 1e-8
    wd: float = 0.0
    lam: float = 0.0
    lam_ramp: int = 0
    opt: int = 0            # 0 Adam, 1 RMSprop, 2 SGD
    momentum: float = 0.0
    rms_alpha: float = 0.99
    dampening: float = 0.0
    manip: int = 0          # 1: manipulated gradients (energies are not formed)
    gamma: float = 1.0      # gamma_grad of the manipulated form
    mdt: int = 0            # 1: neighbours read a bfloat16 copy of the marginals


class Run:
    """Holds one FP64 FEM run: h, m1, m2 and the step counter t."""

    def __init__(self, kind, params: Params, h0, *, n, q=1, u=None, v=None, w=None, off=None, lits=None,
                 node_w=None):
        self.kind, self.p, self.n, self.q = kind, params, n, q
        self.h = _f64(h0).copy()
        self.m1 = np.zeros_like(self.h)
        self.m2 = np.zeros_like(self.h)
        self.t = 0
        self._keep = []
        pb = _Problem()
        pb.kind, pb.n, pb.q, pb.R, pb.T = kind, n, q, params.R, params.T
        pb.sched, pb.lam_ramp = params.sched, int(params.lam_ramp)
        if kind == KIND_MAXSAT:
            off, lits = _i64(off), _i32(lits)
            self._keep += [off, lits]
            pb.ne = off.shape[0] - 1
            pb.off, pb.lits = off.ctypes.data, lits.ctypes.data
        else:
            u, v, w = _i32(u), _i32(v), _f64(w)
            self._keep += [u, v, w]
            pb.ne = u.shape[0]
            pb.eu, pb.ev, pb.w = u.ctypes.data, v.ctypes.data, w.ctypes.data
        pb.beta_min, pb.beta_max, pb.lam = params.beta_min, params.beta_max, params.lam
        pb.lr, pb.b1, pb.b2, pb.eps, pb.wd = params.lr, params.b1, params.b2, params.eps, params.wd
        pb.opt, pb.momentum, pb.rms_alpha, pb.dampening = params.opt, params.momentum, params.rms_alpha, \
            params.dampening
        pb.manip, pb.gamma = int(params.manip), params.gamma
        pb.mdt = int(params.mdt)
        self.node_w = None if node_w is None else _f64(node_w)
        pb.nw = None if self.node_w is None else self.node_w.ctypes.data
        self._pb = pb

    def step(self, n_steps: int, record: bool = False):
        """Advance n_steps; with record, return (g_hist, U_hist, S_hist) of
        the evaluated steps (gradient and energies at h(t) before each
        update)."""
        R = self.p.R
        vals = self.h.size
        gh = np.zeros((n_steps,) + self.h.shape) if record else None
        Uh = np.zeros((n_steps, R)) if record else None
        Sh = np.zeros((n_steps, R)) if record else None
        rc = lib().orc_run(C.byref(self._pb), self.t, n_steps, _p(self.h), _p(self.m1), _p(self.m2),
                           _p(gh), _p(Uh), _p(Sh))
        if rc:
            raise MemoryError(rc)
        assert vals == self.h.size
        self.t += n_steps
        return (gh, Uh, Sh) if record else None

    def sigma(self):
        return round_(self.h, 1 if self.kind != KIND_BMINCUT else self.q)

    def eval_at(self, h, t):
        """(g, U, S) of step t (beta(t), lambda(t)) at fields h, without
        touching the run's own state.  With manipulated gradients U and S are
        None."""
        p = self.p
        b = beta(p.sched, p.beta_min, p.beta_max, p.T, t)
        if p.manip:
            if self.kind == KIND_MAXCUT:
                u, v, w = self._keep
                return maxcut_grad_manip(self.n, u, v, w, h, b, p.gamma), None, None
            if self.kind == KIND_BMINCUT:
                u, v, w = self._keep
                return bmincut_grad_manip(self.n, u, v, w, self.q, lam(p.lam_ramp, p.lam, p.T, t), h, b,
                                          p.gamma, node_w=self.node_w), None, None
            off, lits = self._keep
            return maxsat_grad_manip(self.n, off, lits, h, b, p.gamma), None, None
        if self.kind == KIND_MAXCUT:
            u, v, w = self._keep
            return maxcut_grad(self.n, u, v, w, h, b, mdt=p.mdt)
        if self.kind == KIND_BMINCUT:
            u, v, w = self._keep
            return bmincut_grad(self.n, u, v, w, self.q, lam(p.lam_ramp, p.lam, p.T, t), h, b, node_w=self.node_w,
                                mdt=p.mdt)
        off, lits = self._keep
        return maxsat_grad(self.n, off, lits, h, b, mdt=p.mdt)

    def adam_from(self, h, m1, m2, g, t):
        """Fields after the optimiser step of step t from (h, m1, m2) with
        gradient g (Adam, RMSprop or SGD as the parameters say)."""
        p = self.p
        hh, a, b = (np.array(x, dtype=np.float64, copy=True) for x in (h, m1, m2))
        if p.opt == 1:
            rmsprop(g, hh, a, b, p.lr, p.rms_alpha, p.eps, p.wd, p.momentum)
        elif p.opt == 2:
            sgd(g, hh, a, p.lr, p.wd, p.momentum, p.dampening, t + 1)
        else:
            adam(g, hh, a, b, p.lr, p.b1, p.b2, p.eps, p.wd, t + 1)
        return hh


def maxcut_run(graph, params: Params, h0):
    return Run(KIND_MAXCUT, params, h0, n=graph.n, u=graph.u, v=graph.v, w=graph.w)


def bmincut_run(graph, q, params: Params, h0, node_w=None):
    return Run(KIND_BMINCUT, params, h0, n=graph.n, q=q, u=graph.u, v=graph.v, w=graph.w, node_w=node_w)


def maxsat_run(cnf, params: Params, h0):
    return Run(KIND_MAXSAT, params, h0, n=cnf.n_vars, off=cnf.clause_off, lits=cnf.lits)
