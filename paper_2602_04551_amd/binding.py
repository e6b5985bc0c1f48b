"""ctypes binding of libl0l2 (include/l0l2.h).

Argument marshalling only: every step runs in the HIP library.  torch provides
device memory (tensors on cuda:N) and the stream; nothing here computes the
method.  Importing this module raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libl0l2.so")

L0L2_OK, L0L2_E_INVALID, L0L2_E_NODATA, L0L2_E_OOM = 0, -1, -2, -3
L0L2_E_DEVICE, L0L2_E_NUMERIC, L0L2_E_TIMEOUT, L0L2_E_CANCELLED, L0L2_E_UNSUPPORTED = -4, -5, -6, -7, -8
L0L2_FP64, L0L2_FP32, L0L2_BF16, L0L2_FP8 = 0, 1, 2, 3
L0L2_FREE, L0L2_FIX0, L0L2_FIX1 = 0, 1, 2
L0L2_BEST_FIRST, L0L2_DFS = 0, 1
PRECISIONS = {"fp64": L0L2_FP64, "fp32": L0L2_FP32, "bf16": L0L2_BF16, "fp8": L0L2_FP8}


class l0l2_admm_opts(C.Structure):
    _fields_ = [("tol_node", C.c_double), ("max_iter", C.c_int), ("check_every", C.c_int)]


class l0l2_fista_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int)]


class l0l2_trace_rec(C.Structure):
    _fields_ = [("id", C.c_int64), ("parent", C.c_int64), ("depth", C.c_int32),
                ("branch_j", C.c_int32), ("decision", C.c_int32), ("iters", C.c_int32),
                ("support_size", C.c_int32), ("admm_status", C.c_int32),
                ("lb", C.c_double), ("primal", C.c_double), ("ub_node", C.c_double),
                ("ub_global", C.c_double)]


class l0l2_bnb_opts(C.Structure):
    _fields_ = [("K", C.c_int), ("policy", C.c_int), ("eps_prune", C.c_double),
                ("gap_tol", C.c_double), ("time_limit_s", C.c_double), ("max_nodes", C.c_int64),
                ("max_iter_root", C.c_int), ("admm", l0l2_admm_opts), ("fista", l0l2_fista_opts),
                ("trace", C.POINTER(l0l2_trace_rec)), ("trace_cap", C.c_int64), ("root_heuristic", C.c_int),
                ("init_support", C.c_void_p), ("warm_root", C.c_int)]


class l0l2_bnb_result(C.Structure):
    _fields_ = [("ub", C.c_double), ("certified", C.c_double), ("lb", C.c_double),
                ("nodes_solved", C.c_int64), ("nodes_pruned", C.c_int64), ("trace_len", C.c_int64),
                ("batches", C.c_int64), ("seconds", C.c_double), ("status", C.c_int),
                ("support_len", C.c_int64), ("support", C.POINTER(C.c_int32)),
                ("beta", C.POINTER(C.c_double))]


class l0l2_request_stats(C.Structure):
    _fields_ = [("submit_s", C.c_double), ("admit_s", C.c_double), ("done_s", C.c_double),
                ("footprint_bytes", C.c_size_t), ("peak_bytes", C.c_size_t)]


_vp, _i, _i64, _d = C.c_void_p, C.c_int, C.c_int64, C.c_double
SIGNATURES = {
    "l0l2_create": (_i, [_i, _vp, C.POINTER(_vp)]),
    "l0l2_destroy": (None, [_vp]),
    "l0l2_last_error": (C.c_char_p, [_vp]),
    "l0l2_state_bytes": (_i, [_vp]),
    "l0l2_set_data": (_i, [_vp, _vp, _vp, _i64, _i64, _d, _d, _d, _d, _i, _i]),
    "l0l2_admm_sweeps": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _i]),
    "l0l2_dual_bound": (_i, [_vp, _i, _vp, _vp, _vp]),
    "l0l2_solve_node_batch": (_i, [_vp, _i, _vp, _vp, _vp, C.POINTER(l0l2_admm_opts), _vp, _vp, _vp, _vp]),
    "l0l2_round_branch": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _vp, _vp]),
    "l0l2_solve_node_queue": (_i, [_vp, _i, _vp, _vp, _vp, _i, C.POINTER(l0l2_admm_opts), _vp, _vp, _vp, _vp]),
    "l0l2_batch_stats": (_i, [_vp, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i64)]),
    "l0l2_refine_incumbent": (_i, [_vp, _i, _vp, _vp, _vp, C.POINTER(l0l2_fista_opts), _vp, _vp]),
    "l0l2_refine_incumbent_noalloc": (_i, [_vp, _i, _vp, _vp, _vp, C.POINTER(l0l2_fista_opts), _vp, _vp]),
    "l0l2_exact_objective": (_i, [_vp, _vp, _vp, _vp]),
    "l0l2_matching_pursuit": (_i, [_vp, _i, _vp, _vp, C.POINTER(_d), _vp, C.POINTER(C.c_int32)]),
    "l0l2_bnb_solve": (_i, [_vp, C.POINTER(l0l2_bnb_opts), C.POINTER(l0l2_bnb_result)]),
    "l0l2_result_free": (None, [C.POINTER(l0l2_bnb_result)]),
    "l0l2_footprint_bytes": (C.c_size_t, [_i64, _i64, _i, _i]),
    "l0l2_server_create": (_i, [_i, C.c_size_t, _i, C.POINTER(l0l2_bnb_opts), C.POINTER(_vp)]),
    "l0l2_server_submit": (_i, [_vp, _vp, _vp, _i64, _i64, _d, _d, _d, _d, _i, C.POINTER(_i64)]),
    "l0l2_server_wait": (_i, [_vp, _i64, _d, C.POINTER(l0l2_bnb_result), C.POINTER(l0l2_request_stats)]),
    "l0l2_server_last_error": (C.c_char_p, [_vp]),
    "l0l2_server_destroy": (_i, [_vp]),
    "l0l2_server_cancel": (_i, [_vp, _i64]),
    "l0l2_server_set_batching": (_i, [_vp, _i]),
    "l0l2_server_batching_stats": (_i, [_vp, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i64)]),
    "l0l2_memory_stats": (_i, [_vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t), _i]),
    "l0l2_set_tiles": (_i, [_vp, _i, _i]),
    "l0l2_tune_batch_size": (_i, [_vp, _i, _d, C.POINTER(_i), _vp, C.POINTER(_i)]),
    "l0l2_set_penalties": (_i, [_vp, _d, _d, _d]),
    "l0l2_lambda0_max": (_i, [_vp, C.POINTER(_d)]),
    "l0l2_bnb_path": (_i, [_vp, C.POINTER(l0l2_bnb_opts), _i, _vp, C.POINTER(l0l2_bnb_result)]),
    "l0l2_set_bupdate_form": (_i, [_vp, _i]),
    "l0l2_set_bf16_terms": (_i, [_vp, _i]),
    "l0l2_set_bf16_tile_rows": (_i, [_vp, _i]),
    "l0l2_bupdate_form": (_i, [_vp, C.POINTER(_i), C.POINTER(_d), C.POINTER(_d)]),
    "l0l2_cancel": (_i, [_vp]),
    "l0l2_profile_enable": (_i, [_vp, _i]),
    "l0l2_profile_query": (_i, [_vp, C.c_char_p, C.POINTER(_i64), C.POINTER(_d), C.POINTER(_i64)]),
}


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libl0l2 is not built ({path} missing): run __graft_entry__.build()")
    # torch first: its HIP runtime is then the one the library binds to, the same
    # runtime instance that owns the tensors and streams handed to the library
    # (loaded the other way round, the process can end up with no usable device)
    import torch  # noqa: F401
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = load_library()


class L0L2Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libl0l2 error {code}: {msg}")
        self.code = code


def _torch():
    import torch
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Context:
    """One l0l2_ctx on one device and stream.  Device buffers are torch tensors."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.device = device
        self.torch_device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.torch_device)
        self.stream = stream
        h = C.c_void_p()
        rc = lib.l0l2_create(device, C.c_void_p(stream.cuda_stream), C.byref(h))
        if rc != L0L2_OK:
            raise L0L2Error(rc, lib.l0l2_last_error(None).decode())
        self._h = h
        self.n = self.p = 0
        self.precision = None

    def close(self):
        if getattr(self, "_h", None):
            lib.l0l2_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != L0L2_OK:
            raise L0L2Error(rc, lib.l0l2_last_error(self._h).decode())

    # -- instance ---------------------------------------------------------
    def set_data(self, X, y, lambda0, lambda2, M, rho=1.0, precision="fp64"):
        X = np.asfortranarray(X, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        n, p = X.shape
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self._check(lib.l0l2_set_data(self._h, X.ctypes.data, y.ctypes.data, n, p, float(lambda0),
                                      float(lambda2), float(M), float(rho), prec, 0))
        self.n, self.p, self.precision = n, p, prec
        self.lambda0, self.lambda2, self.M, self.rho = lambda0, lambda2, M, rho

    @property
    def state_dtype(self):
        torch = _torch()
        return torch.float64 if self.precision == L0L2_FP64 else torch.float32

    def _dev(self, a, dtype):
        torch = _torch()
        if isinstance(a, np.ndarray):
            a = torch.from_numpy(np.ascontiguousarray(a))
        return a.to(device=self.torch_device, dtype=dtype).contiguous()

    # -- hot-path entry points ---------------------------------------------
    def admm_sweeps(self, codes, beta, v, sweeps):
        torch = _torch()
        codes = self._dev(codes, torch.uint8)
        K = codes.shape[0]
        beta = self._dev(beta, self.state_dtype).clone()
        v = self._dev(v, self.state_dtype).clone()
        b = torch.empty_like(beta)
        self._check(lib.l0l2_admm_sweeps(self._h, K, _ptr(codes), _ptr(beta), _ptr(v), _ptr(b), int(sweeps)))
        return beta, v, b

    def dual_bound(self, codes, b):
        torch = _torch()
        codes = self._dev(codes, torch.uint8)
        K = codes.shape[0]
        b = self._dev(b, self.state_dtype)
        lb = torch.empty(K, dtype=torch.float64, device=self.torch_device)
        self._check(lib.l0l2_dual_bound(self._h, K, _ptr(codes), _ptr(b), _ptr(lb)))
        return lb

    def solve_node_batch(self, codes, beta=None, v=None, tol_node=1e-6, max_iter=2000, check_every=10):
        torch = _torch()
        codes = self._dev(codes, torch.uint8)
        K = codes.shape[0]
        dt = self.state_dtype
        beta = torch.zeros((K, self.p), dtype=dt, device=self.torch_device) if beta is None else self._dev(beta, dt).clone()
        v = torch.zeros((K, self.p), dtype=dt, device=self.torch_device) if v is None else self._dev(v, dt).clone()
        lb = torch.empty(K, dtype=torch.float64, device=self.torch_device)
        primal = torch.empty_like(lb)
        iters = torch.empty(K, dtype=torch.int32, device=self.torch_device)
        status = torch.empty_like(iters)
        o = l0l2_admm_opts(float(tol_node), int(max_iter), int(check_every))
        self._check(lib.l0l2_solve_node_batch(self._h, K, _ptr(codes), _ptr(beta), _ptr(v), C.byref(o),
                                              _ptr(lb), _ptr(primal), _ptr(iters), _ptr(status)))
        return dict(lb=lb, primal=primal, iters=iters, status=status, beta=beta, v=v)

    def solve_node_queue(self, codes, beta=None, v=None, K=256, tol_node=1e-6, max_iter=2000, check_every=10):
        """N queued nodes through K slots, refilled as nodes retire (l0l2_solve_node_queue)."""
        torch = _torch()
        codes = self._dev(codes, torch.uint8)
        N = codes.shape[0]
        dt = self.state_dtype
        beta = torch.zeros((N, self.p), dtype=dt, device=self.torch_device) if beta is None else self._dev(beta, dt).clone()
        v = torch.zeros((N, self.p), dtype=dt, device=self.torch_device) if v is None else self._dev(v, dt).clone()
        lb = torch.empty(N, dtype=torch.float64, device=self.torch_device)
        primal = torch.empty_like(lb)
        iters = torch.empty(N, dtype=torch.int32, device=self.torch_device)
        status = torch.empty_like(iters)
        o = l0l2_admm_opts(float(tol_node), int(max_iter), int(check_every))
        self._check(lib.l0l2_solve_node_queue(self._h, N, _ptr(codes), _ptr(beta), _ptr(v), int(K), C.byref(o),
                                              _ptr(lb), _ptr(primal), _ptr(iters), _ptr(status)))
        return dict(lb=lb, primal=primal, iters=iters, status=status, beta=beta, v=v)

    def batch_stats(self):
        """(blocks, blocks with < 1/8 of the batch live, live nodes summed over blocks) of the last solve."""
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(lib.l0l2_batch_stats(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def round_branch(self, codes, beta):
        torch = _torch()
        codes = self._dev(codes, torch.uint8)
        K = codes.shape[0]
        beta = self._dev(beta, self.state_dtype)
        sup = torch.empty((K, self.p), dtype=torch.uint8, device=self.torch_device)
        ss = torch.empty(K, dtype=torch.int32, device=self.torch_device)
        bj = torch.empty_like(ss)
        zu = torch.empty_like(ss)
        self._check(lib.l0l2_round_branch(self._h, K, _ptr(codes), _ptr(beta), _ptr(sup), _ptr(ss), _ptr(bj), _ptr(zu)))
        return dict(support=sup, support_size=ss, branch_j=bj, z_up=zu)

    def refine_incumbent(self, support, beta_start, tol=1e-12, max_iter=1000):
        torch = _torch()
        support = self._dev(support, torch.uint8)
        K = support.shape[0]
        start = self._dev(beta_start, self.state_dtype)
        beta = torch.empty((K, self.p), dtype=torch.float64, device=self.torch_device)
        obj = torch.empty(K, dtype=torch.float64, device=self.torch_device)
        iters = torch.empty(K, dtype=torch.int32, device=self.torch_device)
        o = l0l2_fista_opts(float(tol), int(max_iter))
        self._check(lib.l0l2_refine_incumbent(self._h, K, _ptr(support), _ptr(start), _ptr(beta), C.byref(o),
                                              _ptr(obj), _ptr(iters)))
        return obj, beta, iters

    def refine_incumbent_noalloc(self, support, beta_start, beta_out, obj, iters=None, tol=1e-12, max_iter=1000):
        """Allocation-free refinement into caller-provided device tensors
        (beta_out: K x p float64, obj: K float64, iters: K int32 or None)."""
        torch = _torch()
        support = self._dev(support, torch.uint8)
        K = support.shape[0]
        start = self._dev(beta_start, self.state_dtype)
        o = l0l2_fista_opts(float(tol), int(max_iter))
        self._check(lib.l0l2_refine_incumbent_noalloc(self._h, K, _ptr(support), _ptr(start), _ptr(beta_out),
                                                      C.byref(o), _ptr(obj), _ptr(iters)))
        return obj, beta_out, iters

    def exact_objective(self, mask):
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        beta = np.zeros(self.p)
        obj = C.c_double()
        self._check(lib.l0l2_exact_objective(self._h, mask.ctypes.data, beta.ctypes.data, C.byref(obj)))
        return obj.value, beta

    def matching_pursuit(self, max_moves=None):
        """Forward / backward matching pursuit from the empty support:
        (mask, beta, F(S, beta), moves), moves as j + 1 (addition) / -(j + 1) (removal)."""
        if max_moves is None:
            max_moves = 4 * min(self.n, self.p)
        mask = np.zeros(self.p, np.uint8)
        beta = np.zeros(self.p)
        moves = np.zeros(max(int(max_moves), 1), np.int32)
        obj = C.c_double()
        nm = C.c_int32()
        self._check(lib.l0l2_matching_pursuit(self._h, int(max_moves), mask.ctypes.data, beta.ctypes.data,
                                              C.byref(obj), moves.ctypes.data, C.byref(nm)))
        return mask, beta, obj.value, [int(m) for m in moves[:nm.value]]

    def set_penalties(self, lambda0, lambda2=None, M=None):
        """New (lambda0, lambda2, M) for the loaded instance; the precompute is kept."""
        lambda2 = self.lambda2 if lambda2 is None else lambda2
        M = self.M if M is None else M
        self._check(lib.l0l2_set_penalties(self._h, float(lambda0), float(lambda2), float(M)))
        self.lambda0, self.lambda2, self.M = lambda0, lambda2, M

    def lambda0_max(self):
        out = C.c_double()
        self._check(lib.l0l2_lambda0_max(self._h, C.byref(out)))
        return out.value

    def bnb_path(self, lambda0s, K=256, policy="best", tol_node=1e-6, max_iter=2000, max_iter_root=10000,
                 check_every=10, eps_prune=None, gap_tol=0.0, time_limit_s=0.0, max_nodes=10**9,
                 fista_tol=1e-12, fista_max_iter=1000, root_heuristic=False):
        """Branch and bound along the decreasing lambda0 grid, each point warm-started
        from the previous one (its certified support as the first incumbent, its
        root iterates as the root's start): one result dict per grid point."""
        lam = np.ascontiguousarray(lambda0s, dtype=np.float64)
        m = len(lam)
        o = bnb_options(K, policy, tol_node, max_iter, max_iter_root, check_every, eps_prune, gap_tol,
                        time_limit_s, max_nodes, fista_tol, fista_max_iter, root_heuristic)
        res = (l0l2_bnb_result * m)()
        rc = lib.l0l2_bnb_path(self._h, C.byref(o), m, lam.ctypes.data, res)
        try:
            out = [_result_dict(res[i], self.p) for i in range(m) if res[i].support or res[i].beta]
        finally:
            for i in range(m):
                lib.l0l2_result_free(C.byref(res[i]))
        self._check(rc)
        self.lambda0 = float(lam[-1])
        return out

    def tune_batch_size(self, k_max=1024, frac=0.9):
        """(chosen K, {candidate K: node-sweeps per second})."""
        k = C.c_int()
        n = C.c_int()
        rates = np.zeros(12)
        self._check(lib.l0l2_tune_batch_size(self._h, int(k_max), float(frac), C.byref(k), rates.ctypes.data,
                                             C.byref(n)))
        return k.value, {32 << i: float(rates[i]) for i in range(n.value)}

    def set_bupdate_form(self, form="auto"):
        """"auto" (Gram form where it applies), "folded" or "gram"."""
        forms = {"auto": 0, "folded": 1, "gram": 2}
        if form not in forms:
            raise ValueError(f"b-update form must be one of {sorted(forms)}, not {form!r}")
        self._check(lib.l0l2_set_bupdate_form(self._h, forms[form]))

    def memory_stats(self, reset_peak=False):
        """(bytes held now, peak bytes) of the device buffers this context's calls allocated."""
        return memory_stats(self, reset_peak)

    def cancel(self):
        """Ask the running (or next) long call on this context to stop with L0L2_E_CANCELLED."""
        self._check(lib.l0l2_cancel(self._h))

    def bupdate_form(self):
        """("folded" | "gram", measured ms per sweep of the folded form, of the Gram form)."""
        f, a, b = C.c_int(), C.c_double(), C.c_double()
        self._check(lib.l0l2_bupdate_form(self._h, C.byref(f), C.byref(a), C.byref(b)))
        return ("gram" if f.value == 2 else "folded"), a.value, b.value

    def set_bf16_terms(self, terms=1):
        """BF16 Gram-form sweeps: 1 single-term anchored blocks (default), 3 split form in every sweep."""
        self._check(lib.l0l2_set_bf16_terms(self._h, int(terms)))

    def set_bf16_tile_rows(self, rows=128):
        """Rows of the single-term BF16 sweep's largest LDS-staged tile: 128 (default) or 256."""
        self._check(lib.l0l2_set_bf16_tile_rows(self._h, int(rows)))

    def set_tiles(self, xw_shape=-1, xtu_shape=-1):
        self._check(lib.l0l2_set_tiles(self._h, int(xw_shape), int(xtu_shape)))

    def profile_enable(self, enable=True):
        self._check(lib.l0l2_profile_enable(self._h, 1 if enable else 0))

    KERNELS = ("gemm_xw.f32", "admm_xtu.f32", "gemm_xw.f64", "admm_xtu.f64", "gemm_xw.bf16", "admm_xtu.bf16",
               "gap_check", "round_branch", "fista", "anchor.f64", "gemm_xw.fp8", "admm_xtu.fp8")

    def profile_query(self, kernel):
        """(launches, total milliseconds, work units) of one timed kernel family."""
        n, ms, u = C.c_int64(), C.c_double(), C.c_int64()
        self._check(lib.l0l2_profile_query(self._h, kernel.encode(), C.byref(n), C.byref(ms), C.byref(u)))
        return n.value, ms.value, u.value

    def bnb_solve(self, K=256, policy="best", tol_node=1e-6, max_iter=2000, max_iter_root=10000,
                  check_every=10, eps_prune=None, gap_tol=0.0, time_limit_s=0.0, max_nodes=10**9,
                  fista_tol=1e-12, fista_max_iter=1000, trace_cap=0, root_heuristic=False, init_support=None,
                  warm_root=False):
        if eps_prune is None:
            eps_prune = 2.0 * tol_node
        tr = (l0l2_trace_rec * max(trace_cap, 1))()
        o = l0l2_bnb_opts(int(K), L0L2_DFS if policy == "dfs" else L0L2_BEST_FIRST, float(eps_prune),
                          float(gap_tol), float(time_limit_s), int(max_nodes), int(max_iter_root),
                          l0l2_admm_opts(float(tol_node), int(max_iter), int(check_every)),
                          l0l2_fista_opts(float(fista_tol), int(fista_max_iter)),
                          tr if trace_cap > 0 else None, int(trace_cap), 1 if root_heuristic else 0)
        init = None
        if init_support is not None:
            init = np.zeros(self.p, np.uint8)
            init[np.asarray(init_support, dtype=np.int64)] = 1
            o.init_support = init.ctypes.data
        o.warm_root = 1 if warm_root else 0
        r = l0l2_bnb_result()
        self._check(lib.l0l2_bnb_solve(self._h, C.byref(o), C.byref(r)))
        try:
            support = np.array([r.support[i] for i in range(r.support_len)], dtype=np.int64)
            beta = np.ctypeslib.as_array(r.beta, shape=(self.p,)).copy()
        finally:
            lib.l0l2_result_free(C.byref(r))
        n_tr = min(r.trace_len, trace_cap)
        trace = [{f: getattr(tr[i], f) for f, _ in l0l2_trace_rec._fields_} for i in range(n_tr)]
        return dict(ub=r.ub, certified=r.certified, lb=r.lb, nodes_solved=r.nodes_solved,
                    nodes_pruned=r.nodes_pruned, batches=r.batches, seconds=r.seconds, status=r.status,
                    support=support, beta=beta, trace=trace)


def memory_stats(ctx=None, reset_peak=False):
    """(bytes held now, peak bytes) of the library's device buffers: of one
    Context, or of the whole process (ctx None)."""
    a, b = C.c_size_t(), C.c_size_t()
    lib.l0l2_memory_stats(ctx._h if ctx is not None else None, C.byref(a), C.byref(b), 1 if reset_peak else 0)
    return a.value, b.value


def bnb_options(K=256, policy="best", tol_node=1e-6, max_iter=2000, max_iter_root=10000, check_every=10,
                eps_prune=None, gap_tol=0.0, time_limit_s=0.0, max_nodes=10**9, fista_tol=1e-12,
                fista_max_iter=1000, root_heuristic=False):
    if eps_prune is None:
        eps_prune = 2.0 * tol_node
    return l0l2_bnb_opts(int(K), L0L2_DFS if policy == "dfs" else L0L2_BEST_FIRST, float(eps_prune),
                         float(gap_tol), float(time_limit_s), int(max_nodes), int(max_iter_root),
                         l0l2_admm_opts(float(tol_node), int(max_iter), int(check_every)),
                         l0l2_fista_opts(float(fista_tol), int(fista_max_iter)), None, 0,
                         1 if root_heuristic else 0)


def _result_dict(r, p):
    support = np.array([r.support[i] for i in range(r.support_len)], dtype=np.int64)
    beta = np.ctypeslib.as_array(r.beta, shape=(p,)).copy() if r.beta else np.zeros(p)
    return dict(ub=r.ub, certified=r.certified, lb=r.lb, nodes_solved=r.nodes_solved,
                nodes_pruned=r.nodes_pruned, batches=r.batches, seconds=r.seconds, status=r.status,
                support=support, beta=beta)


class Server:
    """l0l2_server: continuous batching of whole branch-and-bound solves."""

    def __init__(self, device=0, hbm_budget_bytes=0, max_concurrent=4, batching=True, **bnb_kw):
        h = C.c_void_p()
        self.opts = bnb_options(**bnb_kw)
        rc = lib.l0l2_server_create(device, int(hbm_budget_bytes), int(max_concurrent), C.byref(self.opts),
                                    C.byref(h))
        if rc != L0L2_OK:
            raise L0L2Error(rc, "server creation failed")
        self._h = h
        self._p = {}
        self.set_batching(batching)

    def set_batching(self, on):
        rc = lib.l0l2_server_set_batching(self._h, 1 if on else 0)
        if rc != L0L2_OK:
            raise L0L2Error(rc, "set_batching failed")

    def batching_stats(self):
        """Executor counters: rounds, blocks, grouped launches, instance
        contractions carried by them."""
        v = [C.c_int64() for _ in range(4)]
        rc = lib.l0l2_server_batching_stats(self._h, *[C.byref(x) for x in v])
        if rc != L0L2_OK:
            raise L0L2Error(rc, "batching_stats failed")
        return dict(rounds=v[0].value, blocks=v[1].value, launches=v[2].value, members=v[3].value)

    def submit(self, X, y, lambda0, lambda2, M, rho=1.0, precision="fp32"):
        X = np.asfortranarray(X, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        n, p = X.shape
        rid = C.c_int64()
        rc = lib.l0l2_server_submit(self._h, X.ctypes.data, y.ctypes.data, n, p, float(lambda0), float(lambda2),
                                    float(M), float(rho), PRECISIONS[precision], C.byref(rid))
        if rc != L0L2_OK:
            raise L0L2Error(rc, lib.l0l2_server_last_error(self._h).decode())
        self._p[rid.value] = p
        return rid.value

    def wait(self, rid, timeout_s=-1.0):
        r = l0l2_bnb_result()
        st = l0l2_request_stats()
        rc = lib.l0l2_server_wait(self._h, int(rid), float(timeout_s), C.byref(r), C.byref(st))
        if rc == L0L2_E_CANCELLED:
            # the server may be being destroyed by another thread: do not call into it again
            raise L0L2Error(rc, "request cancelled")
        if rc != L0L2_OK:
            raise L0L2Error(rc, lib.l0l2_server_last_error(self._h).decode())
        try:
            out = _result_dict(r, self._p.pop(rid))
        finally:
            lib.l0l2_result_free(C.byref(r))
        out.update(submit_s=st.submit_s, admit_s=st.admit_s, done_s=st.done_s,
                   footprint_bytes=st.footprint_bytes, peak_bytes=st.peak_bytes)
        return out

    def cancel(self, rid):
        rc = lib.l0l2_server_cancel(self._h, int(rid))
        if rc != L0L2_OK:
            raise L0L2Error(rc, "unknown or collected request")

    def close(self):
        if getattr(self, "_h", None):
            lib.l0l2_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
