"""ctypes wrapper around the plain FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The HIP library never loads it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC = os.path.join(_HERE, "l0l2_oracle.c")

FREE, FIX0, FIX1 = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
                               SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)   # a process that has the old library loaded keeps it
    return LIB_PATH


class TraceRec(C.Structure):
    _fields_ = [("id", C.c_int64), ("parent", C.c_int64), ("depth", C.c_int32),
                ("branch_j", C.c_int32), ("decision", C.c_int32), ("iters", C.c_int32),
                ("support_size", C.c_int32), ("admm_status", C.c_int32),
                ("lb", C.c_double), ("primal", C.c_double), ("ub_node", C.c_double),
                ("ub_global", C.c_double)]


class BnbOpts(C.Structure):
    _fields_ = [("tol_node", C.c_double), ("max_iter", C.c_int), ("max_iter_root", C.c_int),
                ("check_every", C.c_int), ("eps_prune", C.c_double), ("gap_tol", C.c_double),
                ("max_nodes", C.c_int64), ("fista_tol", C.c_double), ("fista_max_iter", C.c_int)]


class BnbResult(C.Structure):
    _fields_ = [("ub", C.c_double), ("certified", C.c_double), ("lb_global", C.c_double),
                ("nodes_solved", C.c_int64), ("nodes_pruned", C.c_int64), ("trace_len", C.c_int64),
                ("status", C.c_int)]


_lib = None
_D = C.POINTER(C.c_double)
_U8 = C.POINTER(C.c_uint8)


def lib():
    global _lib
    if _lib is None:
        build()   # compiles when the library is missing or older than its source
        L = C.CDLL(LIB_PATH)
        d, i, i64, vp = C.c_double, C.c_int, C.c_int64, C.c_void_p
        for name, res, args in [
            ("orc_T", d, [d, d, d]), ("orc_psi", d, [d, i, d, d, d]),
            ("orc_prox", d, [d, i, d, d, d, d]), ("orc_h", d, [d, d, d, d]),
            ("orc_nu", d, [d, i, d, d, d]), ("orc_z", d, [d, i, d, d, d]),
            ("orc_create", vp, [_D, _D, i64, i64, d, d, d, d]), ("orc_free", None, [vp]),
            ("orc_create_factored", vp, [_D, _D, i64, i64, d, d, d, d, _D]),
            ("orc_c", _D, [vp]),
            ("orc_b_update", None, [vp, _D, _D]),
            ("orc_admm_sweep", None, [vp, _U8, _D, _D, _D]),
            ("orc_primal", d, [vp, _U8, _D]), ("orc_dual_value", d, [vp, _U8, _D]),
            ("orc_dual_bound", d, [vp, _U8, _D]),
            ("orc_node_admm", i, [vp, _U8, _D, _D, _D, d, i, i, _D, _D, C.POINTER(C.c_int)]),
            ("orc_support", i, [vp, _U8, _D, _U8]), ("orc_branch", i, [vp, _U8, _D]),
            ("orc_fista", d, [vp, _U8, _D, d, i, C.POINTER(C.c_int)]),
            ("orc_exact_objective", d, [vp, _U8, _D]), ("orc_objective", d, [vp, _U8, _D]),
            ("orc_bnb", i, [vp, C.POINTER(BnbOpts), C.POINTER(BnbResult), _U8, _D,
                            C.POINTER(TraceRec), i64]),
            ("orc_mp_deltas", None, [vp, _U8, _D, _D, _D, _D]),
            ("orc_matching_pursuit", i, [vp, i, _U8, _D, C.POINTER(C.c_int32)]),
        ]:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _up(a):
    return a.ctypes.data_as(_U8)


def T(t, a, m):
    return lib().orc_T(t, a, m)


def psi(beta, code, l0, l2, M):
    return lib().orc_psi(beta, code, l0, l2, M)


def prox(bt, code, l0, l2, M, rho):
    return lib().orc_prox(bt, code, l0, l2, M, rho)


def h(x, l0, l2, M):
    return lib().orc_h(x, l0, l2, M)


def nu(x, code, l0, l2, M):
    return lib().orc_nu(x, code, l0, l2, M)


def z(beta, code, l0, l2, M):
    return lib().orc_z(beta, code, l0, l2, M)


class Oracle:
    """One problem instance held by the oracle (X, y, lambda0, lambda2, M, rho)."""

    def __init__(self, X, y, lambda0, lambda2, M, rho=1.0, factor=None):
        """factor=None: the oracle forms the once-per-tree factor itself (plain C
        loops, O(n p min(n, p)) single-threaded).  factor="numpy": the factor is
        taken from numpy's LAPACK routines instead (for the large instances;
        only that precompute differs)."""
        X = np.asfortranarray(X, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        self.n, self.p = X.shape
        self.lambda0, self.lambda2, self.M, self.rho = float(lambda0), float(lambda2), float(M), float(rho)
        self.X, self.y = X, y
        if factor is None:
            self._h = lib().orc_create(_dp(X), _dp(y), self.n, self.p, self.lambda0, self.lambda2,
                                       self.M, self.rho)
        elif factor == "numpy":
            if self.n >= self.p:
                A = X.T @ X + self.rho * np.eye(self.p)
                F = np.asfortranarray(np.linalg.inv(A))
            else:
                F = np.asfortranarray(np.linalg.cholesky(X @ X.T + self.rho * np.eye(self.n)))
            self._h = lib().orc_create_factored(_dp(X), _dp(y), self.n, self.p, self.lambda0, self.lambda2,
                                                self.M, self.rho, _dp(F))
        else:
            raise ValueError("factor is None or 'numpy'")
        if not self._h:
            raise ValueError("oracle rejected the instance")

    @classmethod
    def from_instance(cls, inst, rho=1.0, factor=None):
        return cls(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, rho, factor=factor)

    def __del__(self):
        h_ = getattr(self, "_h", None)
        if h_:
            lib().orc_free(h_)
            self._h = None

    def _codes(self, codes):
        c = np.zeros(self.p, np.uint8) if codes is None else np.ascontiguousarray(codes, np.uint8)
        assert c.shape == (self.p,)
        return c

    @property
    def c(self):
        ptr = lib().orc_c(self._h)
        return np.ctypeslib.as_array(ptr, shape=(self.p,)).copy()

    def b_update(self, w):
        w = np.ascontiguousarray(w, np.float64)
        b = np.empty(self.p)
        lib().orc_b_update(self._h, _dp(w), _dp(b))
        return b

    def sweep(self, codes, beta, v):
        """One ADMM sweep; returns new (beta, v, b) without touching the inputs."""
        c = self._codes(codes)
        beta = np.array(beta, np.float64)
        v = np.array(v, np.float64)
        b = np.empty(self.p)
        lib().orc_admm_sweep(self._h, _up(c), _dp(beta), _dp(v), _dp(b))
        return beta, v, b

    def primal(self, codes, beta):
        return lib().orc_primal(self._h, _up(self._codes(codes)), _dp(np.ascontiguousarray(beta, np.float64)))

    def dual_value(self, codes, r):
        return lib().orc_dual_value(self._h, _up(self._codes(codes)), _dp(np.ascontiguousarray(r, np.float64)))

    def dual_bound(self, codes, r):
        return lib().orc_dual_bound(self._h, _up(self._codes(codes)), _dp(np.ascontiguousarray(r, np.float64)))

    def node_admm(self, codes, beta=None, v=None, tol=1e-6, max_iter=2000, check_every=10):
        """Solve one node relaxation; returns dict(lb, primal, iters, status, beta, v, b)."""
        c = self._codes(codes)
        beta = np.zeros(self.p) if beta is None else np.array(beta, np.float64)
        v = np.zeros(self.p) if v is None else np.array(v, np.float64)
        b = np.zeros(self.p)
        lb, pr, it = C.c_double(), C.c_double(), C.c_int()
        st = lib().orc_node_admm(self._h, _up(c), _dp(beta), _dp(v), _dp(b), tol, max_iter,
                                 check_every, C.byref(lb), C.byref(pr), C.byref(it))
        return dict(lb=lb.value, primal=pr.value, iters=it.value, status=st, beta=beta, v=v, b=b)

    def support(self, codes, beta):
        m = np.zeros(self.p, np.uint8)
        k = lib().orc_support(self._h, _up(self._codes(codes)), _dp(np.ascontiguousarray(beta, np.float64)), _up(m))
        return m, k

    def branch(self, codes, beta):
        return lib().orc_branch(self._h, _up(self._codes(codes)), _dp(np.ascontiguousarray(beta, np.float64)))

    def fista(self, mask, beta0, tol=1e-12, max_iter=1000):
        m = np.ascontiguousarray(mask, np.uint8)
        b = np.array(beta0, np.float64)
        it = C.c_int()
        f = lib().orc_fista(self._h, _up(m), _dp(b), tol, max_iter, C.byref(it))
        return f, b, it.value

    def exact_objective(self, mask):
        m = np.ascontiguousarray(mask, np.uint8)
        b = np.zeros(self.p)
        f = lib().orc_exact_objective(self._h, _up(m), _dp(b))
        return f, b

    def objective(self, mask, beta):
        return lib().orc_objective(self._h, _up(np.ascontiguousarray(mask, np.uint8)),
                                   _dp(np.ascontiguousarray(beta, np.float64)))

    def mp_deltas(self, mask, beta, r):
        """Objective change of every single-coordinate move (App. A.2) and the
        coefficient each move sets."""
        delta = np.empty(self.p)
        bnew = np.empty(self.p)
        lib().orc_mp_deltas(self._h, _up(np.ascontiguousarray(mask, np.uint8)),
                            _dp(np.ascontiguousarray(beta, np.float64)), _dp(np.ascontiguousarray(r, np.float64)),
                            _dp(delta), _dp(bnew))
        return delta, bnew

    def matching_pursuit(self, max_moves=None):
        """Forward / backward matching pursuit from the empty support: (mask, beta, moves)."""
        if max_moves is None:
            max_moves = 4 * self.p
        mask = np.zeros(self.p, np.uint8)
        beta = np.zeros(self.p)
        moves = np.zeros(max(max_moves, 1), np.int32)
        nm = lib().orc_matching_pursuit(self._h, int(max_moves), _up(mask), _dp(beta),
                                        moves.ctypes.data_as(C.POINTER(C.c_int32)))
        return mask, beta, [int(m) for m in moves[:nm]]

    def bnb(self, tol_node=1e-6, max_iter=2000, max_iter_root=10000, check_every=10,
            eps_prune=None, gap_tol=0.0, max_nodes=10**7, fista_tol=1e-12, fista_max_iter=1000,
            trace_cap=100000):
        if eps_prune is None:
            eps_prune = 2.0 * tol_node
        o = BnbOpts(tol_node, max_iter, max_iter_root, check_every, eps_prune, gap_tol, max_nodes,
                    fista_tol, fista_max_iter)
        r = BnbResult()
        mask = np.zeros(self.p, np.uint8)
        beta = np.zeros(self.p)
        tr = (TraceRec * max(trace_cap, 1))()
        lib().orc_bnb(self._h, C.byref(o), C.byref(r), _up(mask), _dp(beta), tr, trace_cap)
        n_tr = min(r.trace_len, trace_cap)
        trace = [{f: getattr(tr[i], f) for f, _ in TraceRec._fields_} for i in range(n_tr)]
        return dict(ub=r.ub, certified=r.certified, lb_global=r.lb_global,
                    nodes_solved=r.nodes_solved, nodes_pruned=r.nodes_pruned, status=r.status,
                    support=np.flatnonzero(mask), mask=mask, beta=beta, trace=trace)
