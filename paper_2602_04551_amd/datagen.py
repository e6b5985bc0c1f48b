"""Seeded synthetic instances for the l0-l2 regression problem.

This module only draws inputs: the design matrix X, the response y and the
problem parameters (lambda0, lambda2, M).  It holds none of the method's
arithmetic and is imported both by the tests that drive the CPU oracle and by
the HIP path's benchmark, so the two sides always see the same bytes.

Recipe (Sec. 4.1, synthetic datasets, with the concrete correlation models of
the workloads in use):

* rows of X are N(0, Sigma).  Two Sigma families are used:
  - Toeplitz, Sigma_ij = rho_T^|i-j|: generated column by column with the
    exact AR(1) recursion x_0 = xi_0, x_j = rho_T x_{j-1} + sqrt(1-rho_T^2) xi_j;
  - constant correlation, Sigma = rho_c 11^T + (1-rho_c) I (the paper's own
    family): x_j = sqrt(rho_c) omega + sqrt(1-rho_c) xi_j with a shared omega;
* columns are centred and scaled to unit Euclidean norm;
* beta_dagger has k unit entries at the equispaced indices floor(j p / k);
* y = X beta_dagger + eps, eps ~ N(0, sigma^2 I), sigma^2 = Var(X beta_dagger) / SNR
  (population variance over the n samples);
* y is centred and scaled to unit norm.

M follows the paper's rule M = 1.5 M* with M* the largest magnitude of the ridge
fit restricted to the true support (Sec. 4.1, selection of lambda0, lambda2, M).
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = ["Instance", "make_instance", "CONFIGS", "config_instance", "node_batch_codes", "frontier_codes",
           "select_lambda2", "node_parallel_instance", "serving_instance", "FREE", "FIX0", "FIX1"]

FREE, FIX0, FIX1 = 0, 1, 2


@dataclasses.dataclass
class Instance:
    X: np.ndarray          # (n, p) float64, Fortran (column-major) order
    y: np.ndarray          # (n,) float64
    lambda0: float
    lambda2: float
    M: float
    beta_true: np.ndarray  # (p,) float64
    name: str = ""
    seed: int = 0
    y_scale: float = 1.0   # the norm y was divided by: the truth in the units of y is beta_true / y_scale

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def p(self) -> int:
        return self.X.shape[1]


def _design(rng: np.random.Generator, n: int, p: int, corr: str, rho: float) -> np.ndarray:
    X = np.empty((n, p), dtype=np.float64, order="F")
    if corr == "toeplitz":
        s = np.sqrt(1.0 - rho * rho)
        X[:, 0] = rng.standard_normal(n)
        for j in range(1, p):
            X[:, j] = rho * X[:, j - 1] + s * rng.standard_normal(n)
    elif corr == "constant":
        omega = rng.standard_normal(n)
        a, b = np.sqrt(rho), np.sqrt(1.0 - rho)
        for j in range(p):
            X[:, j] = a * omega + b * rng.standard_normal(n)
    else:
        raise ValueError(f"unknown correlation model {corr!r}")
    X -= X.mean(axis=0, keepdims=True)
    nrm = np.linalg.norm(X, axis=0)
    nrm[nrm == 0.0] = 1.0
    X /= nrm
    return np.asfortranarray(X)


def _ridge_on_support(X: np.ndarray, y: np.ndarray, support: np.ndarray, lambda2: float) -> np.ndarray:
    XS = X[:, support]
    A = XS.T @ XS + 2.0 * lambda2 * np.eye(len(support))
    return np.linalg.solve(A, XS.T @ y)


def make_instance(n: int, p: int, *, corr: str = "toeplitz", rho: float = 0.5, k: int = 10,
                  snr: float = 5.0, lambda0: float = 0.005, lambda2: float = 0.01,
                  M: float | None = None, seed: int = 0, name: str = "") -> Instance:
    """Draw one instance.  M=None applies the 1.5 x ridge-on-true-support rule."""
    if n < 1 or p < 1 or k < 0 or k > p:
        raise ValueError("need n>=1, p>=1, 0<=k<=p")
    rng = np.random.default_rng(seed)
    X = _design(rng, n, p, corr, rho)
    beta = np.zeros(p)
    support = np.array([(j * p) // k for j in range(k)], dtype=np.int64) if k else np.zeros(0, np.int64)
    beta[support] = 1.0
    signal = X @ beta
    var = float(np.var(signal)) if k else 0.0
    sigma = np.sqrt(var / snr) if var > 0 else 1.0
    y = signal + sigma * rng.standard_normal(n)
    y -= y.mean()
    ny = np.linalg.norm(y)
    if ny > 0:
        y /= ny
    if M is None:
        M = 1.5 * float(np.max(np.abs(_ridge_on_support(X, y, support, lambda2)))) if k else 1.0
    return Instance(X=X, y=y, lambda0=float(lambda0), lambda2=float(lambda2), M=float(M),
                    beta_true=beta, name=name, seed=seed, y_scale=float(ny) if ny > 0 else 1.0)


# The workloads: (small oracle case, plain GPU case, batching, serving draw, high-dim).
CONFIGS = {
    "C1": dict(n=100, p=50, corr="toeplitz", rho=0.1, k=5, snr=5.0, lambda0=0.01, lambda2=0.01),
    "C2": dict(n=1000, p=1000, corr="toeplitz", rho=0.5, k=10, snr=5.0, lambda0=0.005, lambda2=0.01),
    "C3": dict(n=5000, p=5000, corr="toeplitz", rho=0.3, k=20, snr=3.0, lambda0=0.005, lambda2=0.01),
    "C5": dict(n=1000, p=50000, corr="constant", rho=0.2, k=25, snr=3.0, lambda0=0.002, lambda2=0.005),
}


def config_instance(name: str, seed: int = 0, **override) -> Instance:
    kw = dict(CONFIGS[name])
    kw.update(override)
    return make_instance(seed=seed, name=name, **kw)


def select_lambda2(inst: Instance, grid=None) -> float:
    """lambda2* of Sec. 4.1: the lambda2 on a grid (100 log-spaced points over
    [1e-4, 1e4]) whose ridge fit restricted to the true support is closest in
    l2 to beta_dagger, taken in the units of the scaled response (beta_dagger /
    y_scale: y was divided by its norm)."""
    grid = np.logspace(-4, 4, 100) if grid is None else np.asarray(grid, dtype=np.float64)
    support = np.flatnonzero(inst.beta_true)
    if len(support) == 0:
        return float(grid[0])
    truth = inst.beta_true[support] / inst.y_scale
    errs = [np.linalg.norm(_ridge_on_support(inst.X, inst.y, support, l2) - truth) for l2 in grid]
    return float(grid[int(np.argmin(errs))])


def node_parallel_instance(p: int, seed: int = 0) -> Instance:
    """The node-parallel study's design (Sec. 4.4, with the data of Sec. 4.1):
    n = 3000, constant correlation 0.2, k = 10 unit spikes, SNR = 10/3; lambda2 =
    lambda2* (select_lambda2), M = 1.5 x the ridge fit on the true support at
    that lambda2.  lambda0 is left to the caller (the paper tunes it along a
    path); the placeholder is 0.005."""
    inst = make_instance(3000, p, corr="constant", rho=0.2, k=10, snr=10.0 / 3.0, lambda0=0.005,
                         lambda2=0.01, seed=seed, name=f"np{p}")
    l2 = select_lambda2(inst)
    support = np.flatnonzero(inst.beta_true)
    inst.lambda2 = l2
    inst.M = 1.5 * float(np.max(np.abs(_ridge_on_support(inst.X, inst.y, support, l2))))
    return inst


def serving_instance(rng: np.random.Generator, seed: int) -> Instance:
    """One draw of the serving stream: n~U{500..5000}, p~U{1000..20000}, rho_T~U[0,0.7],
    k~U{5..30}, SNR~U[2,10], lambda2=0.01, lambda0=0.005."""
    n = int(rng.integers(500, 5001))
    p = int(rng.integers(1000, 20001))
    return make_instance(n, p, corr="toeplitz", rho=float(rng.uniform(0.0, 0.7)),
                         k=int(rng.integers(5, 31)), snr=float(rng.uniform(2.0, 10.0)),
                         lambda0=0.005, lambda2=0.01, seed=seed, name="serve")


def node_batch_codes(p: int, K: int, *, seed: int = 0, free_min: int = 50, free_max: int | None = None,
                     fix1_max: int = 20, keep_free: np.ndarray | None = None) -> np.ndarray:
    """K synthetic BnB nodes as a (K, p) uint8 array of fixing codes.

    Node k keeps f ~ U{free_min..free_max} coordinates free (uniformly random
    positions), fixes |F1| ~ U{0..fix1_max} of the others to one and the rest to
    zero.  Coordinates listed in keep_free are never fixed to zero (so the
    planted support stays reachable)."""
    rng = np.random.default_rng(seed)
    free_max = p if free_max is None else min(free_max, p)
    free_min = min(free_min, free_max)
    codes = np.full((K, p), FIX0, dtype=np.uint8)
    for k in range(K):
        f = int(rng.integers(free_min, free_max + 1))
        perm = rng.permutation(p)
        if keep_free is not None and len(keep_free):
            kf = np.asarray(keep_free)
            perm = np.concatenate([kf, np.setdiff1d(perm, kf, assume_unique=False)[rng.permutation(p - len(kf))]])
        free = perm[:f]
        rest = perm[f:]
        n1 = int(rng.integers(0, min(fix1_max, len(rest)) + 1)) if len(rest) else 0
        codes[k, free] = FREE
        codes[k, rest[:n1]] = FIX1
    return codes


def frontier_codes(p: int, K: int, candidates, *, seed: int = 0, depth_min: int = 1,
                   depth_max: int = 16) -> np.ndarray:
    """K synthetic best-first frontier nodes as a (K, p) uint8 array of codes.

    Node k fixes d ~ U{depth_min..depth_max} distinct coordinates drawn from
    `candidates` (the coordinates a tree near the root branches on), each to
    z = 0 or z = 1 with probability 1/2; every other coordinate is free."""
    rng = np.random.default_rng(seed)
    cand = np.asarray(candidates, dtype=np.int64)
    codes = np.zeros((K, p), dtype=np.uint8)
    for k in range(K):
        d = int(rng.integers(depth_min, min(depth_max, len(cand)) + 1))
        idx = rng.choice(cand, size=d, replace=False)
        codes[k, idx] = rng.choice([FIX0, FIX1], size=d)
    return codes
