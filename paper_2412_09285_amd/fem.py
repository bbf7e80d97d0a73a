"""Thin Python binding of the FEM C ABI (``include/fem.h``).

Argument marshalling only: every step of the hot path runs in the HIP
library ``libfem.so``.  NumPy arrays are passed as host pointers; torch tensors
on the GPU are passed as device pointers (``on_device = 1``).  Streams are
taken from torch (``torch.cuda.current_stream().cuda_stream``) when torch is
used, else the null stream.

If the library has not been built, loading fails loudly: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfem.so")

FEM_OK, FEM_E_INVAL, FEM_E_NOMEM, FEM_E_HIP, FEM_E_STATE, FEM_E_NUMERIC, FEM_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
MAXCUT, BMINCUT, MAXSAT = 0, 1, 2
SCHED_LINEAR, SCHED_EXP, SCHED_INVPROP = 0, 1, 2
OPT_ADAM, OPT_RMSPROP, OPT_SGD = 0, 1, 2
GRAD_EXPLICIT, GRAD_MANIPULATED = 0, 1
STATE_SEPARATE, STATE_INTERLEAVED = 0, 1
F32, BF16 = 0, 1
# size of the per-device scratch array of fem_eval_int_noalloc (FEM_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20


class FemError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_str(status)}: {message}")
        self.status = status
        self.message = message


class Params(C.Structure):
    _fields_ = [
        ("replicas", C.c_int32), ("steps", C.c_int32), ("schedule", C.c_int32),
        ("beta_min", C.c_double), ("beta_max", C.c_double),
        ("lr", C.c_double), ("adam_b1", C.c_double), ("adam_b2", C.c_double),
        ("adam_eps", C.c_double), ("weight_decay", C.c_double),
        ("lam", C.c_double), ("lambda_ramp", C.c_int32),
        ("marginal_dtype", C.c_int32), ("energy_every", C.c_int32),
        ("record_energies", C.c_int32), ("eval_every", C.c_int32), ("keep_grad", C.c_int32),
        ("optimizer", C.c_int32), ("momentum", C.c_double), ("rms_alpha", C.c_double), ("dampening", C.c_double),
        ("gradient", C.c_int32), ("gamma_grad", C.c_double), ("state_layout", C.c_int32),
    ]


class Tile(C.Structure):
    _fields_ = [("vec", C.c_int32), ("waves", C.c_int32), ("rows", C.c_int32), ("nt", C.c_int32),
                ("lanes", C.c_int32)]


_lib = None
_P = C.c_void_p
_PP = C.POINTER(C.c_void_p)

# name -> (restype, argtypes)
_SIGS = {
    "fem_status_str": (C.c_char_p, [C.c_int]),
    "fem_last_error": (C.c_char_p, []),
    "fem_abi_version": (C.c_int32, []),
    "fem_maxcut_create": (C.c_int, [C.c_int, C.c_int32, C.c_int64, _P, _P, _P, _PP]),
    "fem_bmincut_create": (C.c_int, [C.c_int, C.c_int32, C.c_int64, _P, _P, _P, C.c_int32, _PP]),
    "fem_maxcut_create_dense": (C.c_int, [C.c_int, C.c_int32, _P, _PP]),
    "fem_bmincut_create_weighted": (C.c_int, [C.c_int, C.c_int32, C.c_int64, _P, _P, _P, C.c_int32, _P, _PP]),
    "fem_maxsat_create": (C.c_int, [C.c_int, C.c_int32, C.c_int64, _P, _P, _PP]),
    "fem_batch_create": (C.c_int, [C.c_int32, _P, _PP]),
    "fem_graph_order": (C.c_int, [C.c_int32, C.c_int64, _P, _P, _P]),
    "fem_problem_info": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "fem_problem_instance_offsets": (C.c_int, [_P, _P]),
    "fem_problem_destroy": (None, [_P]),
    "fem_params_default": (None, [C.POINTER(Params)]),
    "fem_solver_create": (C.c_int, [_P, C.POINTER(Params), _P, _PP]),
    "fem_solver_destroy": (None, [_P]),
    "fem_set_fields": (C.c_int, [_P, _P, C.c_int]),
    "fem_set_adam_state": (C.c_int, [_P, _P, _P, _P, C.c_int32, C.c_int]),
    "fem_step": (C.c_int, [_P, C.c_int32]),
    "fem_run": (C.c_int, [_P]),
    "fem_run_until": (C.c_int, [_P, C.c_int32]),
    "fem_capture": (C.c_int, [_P, C.c_int32]),
    "fem_sync": (C.c_int, [_P]),
    "fem_get_step": (C.c_int, [_P, _P]),
    "fem_get_fields": (C.c_int, [_P, _P, C.c_int]),
    "fem_last_grad": (C.c_int, [_P, _P, C.c_int]),
    "fem_energies": (C.c_int, [_P, _P, _P, _P]),
    "fem_energy_history": (C.c_int, [_P, C.c_int32, C.c_int32, _P, _P, _P]),
    "fem_round": (C.c_int, [_P, _P]),
    "fem_eval_int": (C.c_int, [_P, C.c_int32, _P, _P, _P]),
    "fem_eval_int_noalloc": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P]),
    "fem_best": (C.c_int, [_P, _P, _P, _P]),
    "fem_anytime_best": (C.c_int, [_P, _P]),
    "fem_state_size": (C.c_int, [_P, _P]),
    "fem_get_state": (C.c_int, [_P, _P, C.c_size_t]),
    "fem_set_state": (C.c_int, [_P, _P, C.c_size_t]),
    "fem_get_tile": (C.c_int, [_P, C.POINTER(Tile)]),
    "fem_set_tile": (C.c_int, [_P, C.POINTER(Tile)]),
    "fem_tune": (C.c_int, [_P, C.c_int32, C.c_int32, C.POINTER(Tile)]),
    "fem_mpnn_create": (C.c_int, [C.c_int, _P, C.c_int32, _PP]),
    "fem_mpnn_destroy": (None, [_P]),
    "fem_mpnn_get_params": (C.c_int, [_P, _P]),
    "fem_mpnn_set_params": (C.c_int, [_P, _P]),
    "fem_mpnn_forward": (C.c_int, [_P, _P, _P, C.c_uint64, C.c_int32, _P, C.c_int]),
    "fem_mpnn_train_step": (C.c_int, [_P, _P, _P, _P, C.c_uint64, C.c_int32, C.c_double, _P, _P]),
    "fem_mpnn_infer": (C.c_int, [_P, _P, C.c_int32, _P, C.c_uint64, C.c_float, _P, C.c_int]),
    "fem_mpnn_infer_async": (C.c_int, [_P, _P, C.c_int32, _P, C.c_uint64, C.c_float, _P, _P]),
    "fem_mpnn_save": (C.c_int, [_P, C.c_char_p]),
    "fem_mpnn_load": (C.c_int, [_P, C.c_char_p]),
    "fem_profile": (C.c_int, [_P, C.c_int32]),
    "fem_profile_result": (C.c_int, [_P, _P, _P]),
}


def lib():
    """Load libfem.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: run __graft_entry__.build() "
                               "or python paper_2412_09285_amd/build.py")
        # PyTorch ships its own HIP runtime under the same soname as the
        # system one that libfem links; whichever is loaded first serves the
        # whole process, and torch cannot use a newer system runtime.  Load
        # torch first so that both use its runtime, whatever the import order.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def status_str(st: int) -> str:
    return lib().fem_status_str(st).decode()


def _check(st: int):
    if st != FEM_OK:
        raise FemError(st, lib().fem_last_error().decode())


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def default_params(**kw) -> Params:
    p = Params()
    lib().fem_params_default(C.byref(p))
    for k, v in kw.items():
        if k == "lambda":
            k = "lam"
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def graph_order(n, u, v):
    """Reverse Cuthill-McKee order of the nodes (see fem.h): order[k] is the
    node to relabel as k."""
    u, pu = _host(u, np.int32)
    v, pv = _host(v, np.int32)
    order = np.empty(n, dtype=np.int32)
    _check(lib().fem_graph_order(n, u.shape[0], pu, pv, order.ctypes.data_as(C.c_void_p)))
    return order


def relabel(order, u, v):
    """Edge lists relabelled by order (node order[k] becomes k)."""
    inv = np.empty_like(order)
    inv[order] = np.arange(order.size, dtype=order.dtype)
    return inv[np.asarray(u)], inv[np.asarray(v)]


class Problem:
    """A device-resident problem (one instance, or a block-diagonal batch)."""

    def __init__(self, handle, keep=()):
        self._h = handle
        self._keep = keep
        info = self.info()
        self.kind, self.n, self.q, self.nnz, self.n_inst = (
            info["kind"], info["n"], info["q"], info["nnz"], info["n_instances"])

    @classmethod
    def maxcut(cls, n, u, v, w=None, device=0):
        u, pu = _host(u, np.int32)
        v, pv = _host(v, np.int32)
        pw = None
        if w is not None:
            w, pw = _host(w, np.float32)
        out = C.c_void_p()
        _check(lib().fem_maxcut_create(device, n, u.shape[0], pu, pv, pw, C.byref(out)))
        return cls(out)

    @classmethod
    def bmincut(cls, n, u, v, w, q, device=0, node_weight=None):
        """node_weight: optional positive integer weight per node (community
        sizes); the balance term then counts summed weights per group."""
        u, pu = _host(u, np.int32)
        v, pv = _host(v, np.int32)
        pw = None
        if w is not None:
            w, pw = _host(w, np.float32)
        out = C.c_void_p()
        if node_weight is None:
            _check(lib().fem_bmincut_create(device, n, u.shape[0], pu, pv, pw, q, C.byref(out)))
        else:
            nw, pn = _host(node_weight, np.int32)
            if nw.shape != (n,):
                raise ValueError(f"node_weight must have shape ({n},), got {nw.shape}")
            _check(lib().fem_bmincut_create_weighted(device, n, u.shape[0], pu, pv, pw, q, pn, C.byref(out)))
        return cls(out)

    @classmethod
    def maxcut_dense(cls, W, device=0):
        """MaxCut on a dense symmetric weight matrix W [n][n] (zero diagonal);
        the explicit-gradient step runs on the matrix cores."""
        W = np.ascontiguousarray(W, dtype=np.float32)
        if W.ndim != 2 or W.shape[0] != W.shape[1]:
            raise ValueError(f"W must be square, got shape {W.shape}")
        out = C.c_void_p()
        _check(lib().fem_maxcut_create_dense(device, W.shape[0], W.ctypes.data_as(C.c_void_p), C.byref(out)))
        return cls(out)

    @classmethod
    def maxsat(cls, n_vars, clause_off, lits, device=0):
        off, po = _host(clause_off, np.int64)
        lt, pl = _host(lits, np.int32)
        out = C.c_void_p()
        _check(lib().fem_maxsat_create(device, n_vars, off.shape[0] - 1, po, pl, C.byref(out)))
        return cls(out)

    @classmethod
    def from_graph(cls, g, kind=MAXCUT, q=2, device=0):
        if kind == MAXCUT:
            return cls.maxcut(g.n, g.u, g.v, g.w, device)
        return cls.bmincut(g.n, g.u, g.v, g.w, q, device)

    @classmethod
    def from_cnf(cls, cnf, device=0):
        return cls.maxsat(cnf.n_vars, cnf.clause_off, cnf.lits, device)

    @classmethod
    def batch(cls, parts):
        arr = (C.c_void_p * len(parts))(*[p._h for p in parts])
        out = C.c_void_p()
        _check(lib().fem_batch_create(len(parts), arr, C.byref(out)))
        return cls(out)

    def info(self):
        k, n, q, ni = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        nnz = C.c_int64()
        _check(lib().fem_problem_info(self._h, C.byref(k), C.byref(n), C.byref(q), C.byref(nnz), C.byref(ni)))
        return dict(kind=k.value, n=n.value, q=q.value, nnz=nnz.value, n_instances=ni.value)

    def instance_offsets(self):
        out = np.zeros(self.n_inst + 1, dtype=np.int32)
        _check(lib().fem_problem_instance_offsets(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def eval_int(self, sigma):
        """sigma [R][n] -> (values [B][R] int64, sizes [B][R][q] int64 or None)."""
        sig, ps = _host(sigma, np.int32)
        R = sig.shape[0]
        vals = np.zeros((self.n_inst, R), dtype=np.int64)
        sizes = np.zeros((self.n_inst, R, self.q), dtype=np.int64) if self.kind == BMINCUT else None
        _check(lib().fem_eval_int(self._h, R, ps, vals.ctypes.data_as(C.c_void_p),
                                  None if sizes is None else sizes.ctypes.data_as(C.c_void_p)))
        return vals, sizes

    def eval_int_noalloc(self, sigma, value, sizes=None, stream=None):
        """Device tensors: sigma int32 [R][n], value int64 [B][R], sizes int64
        [B][R][q] or None; enqueued on stream (torch stream, raw handle, or
        None for the null stream); allocates nothing (fem.h)."""
        R = int(sigma.shape[0])
        for t, shape in ((sigma, (R, self.n)), (value, (self.n_inst, R))) + \
                (((sizes, (self.n_inst, R, self.q)),) if sizes is not None else ()):
            assert t.is_cuda and t.is_contiguous() and tuple(t.shape) == shape, (tuple(t.shape), shape)
        _check(lib().fem_eval_int_noalloc(self._h, R, C.c_void_p(sigma.data_ptr()), C.c_void_p(value.data_ptr()),
                                          None if sizes is None else C.c_void_p(sizes.data_ptr()),
                                          _stream_ptr(stream)))

    def close(self):
        if self._h:
            lib().fem_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """R replicas of FEM on one problem (see fem.h for every call)."""

    def __init__(self, problem: Problem, params: Params | None = None, stream=None, **kw):
        self.problem = problem
        self.params = params if params is not None else default_params(**kw)
        self.R = self.params.replicas
        self.Q = problem.q if problem.kind == BMINCUT else 1
        self.shape = (problem.n, self.R) if self.Q == 1 else (problem.n, self.R, self.Q)
        self._h = C.c_void_p()
        _check(lib().fem_solver_create(problem._h, C.byref(self.params), _stream_ptr(stream), C.byref(self._h)))

    # ---- fields
    def set_fields(self, h):
        if _is_torch(h) and h.is_cuda:
            assert h.dtype.__str__() == "torch.float32" and h.is_contiguous()
            assert tuple(h.shape) == self.shape, (tuple(h.shape), self.shape)
            _check(lib().fem_set_fields(self._h, C.c_void_p(h.data_ptr()), 1))
        else:
            a, pa = _host(h, np.float32)
            assert a.shape == self.shape, (a.shape, self.shape)
            _check(lib().fem_set_fields(self._h, pa, 0))

    def set_adam_state(self, h, m1, m2, t):
        """Host arrays in the layout of h; t = the next step to run."""
        arrs = [_host(x, np.float32) for x in (h, m1, m2)]
        for a, _ in arrs:
            assert a.shape == self.shape, (a.shape, self.shape)
        _check(lib().fem_set_adam_state(self._h, arrs[0][1], arrs[1][1], arrs[2][1], t, 0))

    def fields(self, out=None):
        if out is not None and _is_torch(out) and out.is_cuda:
            _check(lib().fem_get_fields(self._h, C.c_void_p(out.data_ptr()), 1))
            return out
        a = np.empty(self.shape, dtype=np.float32)
        _check(lib().fem_get_fields(self._h, a.ctypes.data_as(C.c_void_p), 0))
        return a

    def last_grad(self):
        a = np.empty(self.shape, dtype=np.float32)
        _check(lib().fem_last_grad(self._h, a.ctypes.data_as(C.c_void_p), 0))
        return a

    # ---- stepping
    def step(self, n=1):
        _check(lib().fem_step(self._h, n))

    def run(self):
        _check(lib().fem_run(self._h))

    def run_until(self, t_end):
        _check(lib().fem_run_until(self._h, t_end))

    def capture(self, t_end):
        _check(lib().fem_capture(self._h, t_end))

    def sync(self):
        _check(lib().fem_sync(self._h))

    @property
    def t(self):
        x = C.c_int32()
        _check(lib().fem_get_step(self._h, C.byref(x)))
        return x.value

    # ---- outputs
    def energies(self):
        B = self.problem.n_inst
        U, S, F = (np.zeros((B, self.R)) for _ in range(3))
        _check(lib().fem_energies(self._h, *(x.ctypes.data_as(C.c_void_p) for x in (U, S, F))))
        return U, S, F

    def energy_history(self, first, count):
        B = self.problem.n_inst
        U, S, F = (np.zeros((count, B, self.R)) for _ in range(3))
        _check(lib().fem_energy_history(self._h, first, count, *(x.ctypes.data_as(C.c_void_p) for x in (U, S, F))))
        return U, S, F

    def round(self):
        s = np.zeros((self.R, self.problem.n), dtype=np.int32)
        _check(lib().fem_round(self._h, s.ctypes.data_as(C.c_void_p)))
        return s

    def best(self):
        B = self.problem.n_inst
        rep = np.zeros(B, dtype=np.int32)
        val = np.zeros(B, dtype=np.int64)
        sig = np.zeros(self.problem.n, dtype=np.int32)
        _check(lib().fem_best(self._h, rep.ctypes.data_as(C.c_void_p), val.ctypes.data_as(C.c_void_p),
                              sig.ctypes.data_as(C.c_void_p)))
        return rep, val, sig

    def anytime_best(self):
        out = np.zeros((self.problem.n_inst, self.R))
        _check(lib().fem_anytime_best(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    # ---- checkpoint
    def get_state(self) -> bytes:
        n = C.c_size_t()
        _check(lib().fem_state_size(self._h, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().fem_get_state(self._h, buf, n.value))
        return buf.raw

    def set_state(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        _check(lib().fem_set_state(self._h, buf, len(data)))

    # ---- tiling
    def tile(self):
        """(vec, waves, rows, nt, lanes)"""
        t = Tile()
        _check(lib().fem_get_tile(self._h, C.byref(t)))
        return (t.vec, t.waves, t.rows, t.nt, t.lanes)

    def set_tile(self, vec, waves, rows, nt=0, lanes=0):
        t = Tile(vec, waves, rows, nt, lanes)
        _check(lib().fem_set_tile(self._h, C.byref(t)))

    def tune(self, trial_steps=5, use_cache=True):
        """Time every valid launch shape; returns the chosen (vec, waves, rows, nt, lanes)."""
        t = Tile()
        _check(lib().fem_tune(self._h, trial_steps, int(use_cache), C.byref(t)))
        return (t.vec, t.waves, t.rows, t.nt, t.lanes)

    # ---- profiling
    def profile(self, on=True):
        _check(lib().fem_profile(self._h, int(on)))

    def profile_result(self):
        ms, n = C.c_double(), C.c_int32()
        _check(lib().fem_profile_result(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def close(self):
        if self._h:
            lib().fem_solver_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


N_MPNN_PARAMS = 9409


class MPNN:
    """The warm-start network (see fem.h): parameters live on the device."""

    def __init__(self, theta0, device=0):
        th, pt = _host(theta0, np.float32)
        assert th.size == N_MPNN_PARAMS
        self._h = C.c_void_p()
        _check(lib().fem_mpnn_create(device, pt, th.size, C.byref(self._h)))

    def params(self):
        out = np.empty(N_MPNN_PARAMS, dtype=np.float32)
        _check(lib().fem_mpnn_get_params(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_params(self, theta):
        th, pt = _host(theta, np.float32)
        _check(lib().fem_mpnn_set_params(self._h, pt))

    def forward(self, problem: Problem, state, seed: int, draw: int):
        """Logits z [n] for one replica's fields state [n] (host)."""
        st, ps = _host(state, np.float32)
        assert st.size == problem.n
        z = np.empty(problem.n, dtype=np.float32)
        _check(lib().fem_mpnn_forward(self._h, problem._h, ps, seed, draw, z.ctypes.data_as(C.c_void_p), 0))
        return z

    def train_step(self, batch: Problem, state, labels, seed: int, draw0: int, lr: float, want_grad=False):
        st, ps = _host(state, np.float32)
        lab, pl = _host(labels, np.int32)
        assert st.size == batch.n and lab.size == batch.n
        loss = C.c_double()
        g = np.empty(N_MPNN_PARAMS, dtype=np.float32) if want_grad else None
        _check(lib().fem_mpnn_train_step(self._h, batch._h, ps, pl, seed, draw0, lr, C.byref(loss),
                                         None if g is None else g.ctypes.data_as(C.c_void_p)))
        return (loss.value, g) if want_grad else loss.value

    def infer(self, problem: Problem, state, seed: int, alpha: float, out=None, stream=None):
        """Proposal alpha * z for every replica of state [n][R] (host array,
        or a device tensor together with a device tensor `out`).  With a
        torch stream (device tensors only) the work is queued on it and the
        call returns without waiting."""
        if _is_torch(state) and state.is_cuda:
            assert out is not None and _is_torch(out) and out.is_cuda
            assert state.is_contiguous() and out.is_contiguous() and state.dtype == out.dtype
            R = state.shape[1]
            if stream is not None:
                _check(lib().fem_mpnn_infer_async(self._h, problem._h, R, C.c_void_p(state.data_ptr()), seed, alpha,
                                                  C.c_void_p(out.data_ptr()), C.c_void_p(stream.cuda_stream)))
            else:
                _check(lib().fem_mpnn_infer(self._h, problem._h, R, C.c_void_p(state.data_ptr()), seed, alpha,
                                            C.c_void_p(out.data_ptr()), 1))
            return out
        assert stream is None, "stream-ordered inference takes device tensors"
        st, ps = _host(state, np.float32)
        st = st.reshape(problem.n, -1)
        h = np.empty_like(st)
        _check(lib().fem_mpnn_infer(self._h, problem._h, st.shape[1], ps, seed, alpha, h.ctypes.data_as(C.c_void_p),
                                    0))
        return h

    def save(self, path):
        _check(lib().fem_mpnn_save(self._h, str(path).encode()))

    def load(self, path):
        _check(lib().fem_mpnn_load(self._h, str(path).encode()))

    def close(self):
        if self._h:
            lib().fem_mpnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
