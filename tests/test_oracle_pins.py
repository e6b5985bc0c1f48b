"""Pins for the CPU oracle: each check comes from outside the oracle's own code
(brute-force minimisation, exact rational arithmetic, numpy/scipy library
routines, closed forms), chosen so that a dropped term, a wrong sign or a
swapped operand in the oracle fails at least one of them.
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.optimize import lsq_linear, minimize_scalar

from paper_2602_04551_amd import datagen

GOLD = os.path.join(os.path.dirname(__file__), "golden")
FREE, FIX0, FIX1 = 0, 1, 2


# ----------------------------------------------------------------------------
# independent brute-force references
# ----------------------------------------------------------------------------

def psi_bf(beta, code, l0, l2, M):
    """min over (z, s) of l0 z + l2 s s.t. beta^2 <= s z, |beta| <= M z, z in [0,1]
    with the node fixings (eq. minzs), by bounded scalar minimisation over z."""
    ab = abs(beta)
    if ab > M * (1 + 1e-15):
        return math.inf
    if code == FIX0:
        return 0.0 if beta == 0.0 else math.inf
    if code == FIX1:
        return l0 + l2 * beta * beta
    if ab == 0.0:
        return 0.0
    lo = ab / M
    f = lambda z: l0 * z + l2 * beta * beta / z
    r = minimize_scalar(f, bounds=(lo, 1.0), method="bounded", options=dict(xatol=1e-13))
    return min(r.fun, f(lo), f(1.0))


def prox_bf(bt, code, l0, l2, M, rho):
    if code == FIX0:
        return 0.0
    g = lambda b: 0.5 * rho * (b - bt) ** 2 + psi_bf(b, code, l0, l2, M)
    grid = np.linspace(-M, M, 801)
    vals = np.array([g(b) for b in grid])
    k = int(np.argmin(vals))
    lo, hi = grid[max(k - 1, 0)], grid[min(k + 1, len(grid) - 1)]
    r = minimize_scalar(g, bounds=(lo, hi), method="bounded", options=dict(xatol=1e-12))
    cands = [r.x, lo, hi, 0.0] + ([M, -M] if abs(bt) > 0 else [])
    return min(cands, key=g)


def conj_bf(x, code, l0, l2, M):
    """sup over |b| <= M of x b - psi(b) (x >= 0), the inner problem of Prop. 1's proof."""
    if code == FIX0:
        return 0.0
    f = lambda b: -(x * b - psi_bf(b, code, l0, l2, M))
    r = minimize_scalar(f, bounds=(0.0, M), method="bounded", options=dict(xatol=1e-13))
    return max(-r.fun, -f(0.0), -f(M))


def box_ridge(X, y, S, l2, M):
    """min over |b|<=M of 1/2||y - X_S b||^2 + l2 ||b||^2 as a bounded least-squares problem."""
    S = list(S)
    if not S:
        return 0.5 * float(y @ y), np.zeros(0)
    XS = X[:, S]
    A = np.vstack([XS, math.sqrt(2 * l2) * np.eye(len(S))])
    rhs = np.concatenate([y, np.zeros(len(S))])
    b = np.linalg.solve(XS.T @ XS + 2 * l2 * np.eye(len(S)), XS.T @ y)
    if np.max(np.abs(b)) > M:
        b = lsq_linear(A, rhs, bounds=(-M, M), method="bvls", tol=1e-15).x
    r = y - XS @ b
    return 0.5 * float(r @ r) + l2 * float(b @ b), b


def enumerate_opt(X, y, l0, l2, M):
    p = X.shape[1]
    vals = []
    for mask in itertools.product([0, 1], repeat=p):
        S = [i for i in range(p) if mask[i]]
        f, _ = box_ridge(X, y, S, l2, M)
        vals.append((f + l0 * len(S), tuple(S)))
    vals.sort()
    return vals


# ----------------------------------------------------------------------------
# scalar pieces
# ----------------------------------------------------------------------------

PARAMS = [  # (l0, l2, M): sqrt(l0/l2) below, at and above M, and M large
    (0.01, 0.01, 10.0), (0.01, 0.01, 0.7), (0.005, 0.01, 2.0), (0.2, 0.05, 1.5),
    (0.001, 0.1, 0.05), (0.02, 0.01, math.sqrt(2.0)),
]


@pytest.mark.parametrize("l0,l2,M", PARAMS)
def test_psi_matches_min_over_z_s(orc, l0, l2, M):
    rng = np.random.default_rng(1)
    for beta in np.concatenate([rng.uniform(-M, M, 25), [0.0, M, -M, math.sqrt(l0 / l2)]]):
        if abs(beta) > M:
            continue
        for code in (FREE, FIX1):
            assert orc.psi(beta, code, l0, l2, M) == pytest.approx(psi_bf(beta, code, l0, l2, M), rel=1e-9, abs=1e-12)
    assert orc.psi(0.0, FIX0, l0, l2, M) == 0.0
    assert math.isinf(orc.psi(0.1 * M, FIX0, l0, l2, M))
    assert math.isinf(orc.psi(1.01 * M, FREE, l0, l2, M))


def test_T_is_box_soft_threshold(orc):
    rng = np.random.default_rng(2)
    for _ in range(40):
        t, a, m = rng.normal() * 2, abs(rng.normal()), abs(rng.normal()) + 0.05
        g = lambda x: 0.5 * (x - t) ** 2 + a * abs(x)
        r = minimize_scalar(g, bounds=(-m, m), method="bounded", options=dict(xatol=1e-12))
        best = min([r.x, -m, m, 0.0], key=g)
        assert orc.T(t, a, m) == pytest.approx(best, abs=1e-7)


@pytest.mark.parametrize("l0,l2,M", PARAMS)
@pytest.mark.parametrize("rho", [1.0, 0.3, 4.0])
def test_prox_matches_brute_force(orc, l0, l2, M, rho):
    rng = np.random.default_rng(3)
    s = math.sqrt(l0 / l2)
    a = 2 * math.sqrt(l0 * l2) / rho
    pts = list(rng.normal(0, 1.5 * M, 10)) + [a + s, -(a + s), a + s + 1e-3, a + s - 1e-3, a, 0.0, 3 * M]
    for bt in pts:
        for code in (FREE, FIX1, FIX0):
            got = orc.prox(bt, code, l0, l2, M, rho)
            want = prox_bf(bt, code, l0, l2, M, rho)
            assert got == pytest.approx(want, abs=2e-7), (bt, code)


def test_prox_golden_free_ridge_branch(orc):
    # tests/golden/prox_free_ridge_branch.txt
    vals = {}
    for line in open(os.path.join(GOLD, "prox_free_ridge_branch.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split("=")
            vals[k.strip()] = float(v)
    got = orc.prox(vals["beta_tilde"], FREE, vals["lambda0"], vals["lambda2"], vals["M"], vals["rho"])
    assert got == pytest.approx(vals["prox"], rel=1e-15)
    assert abs(got - vals["soft_threshold_only"]) > 5e-3


@pytest.mark.parametrize("l0,l2,M", PARAMS)
def test_h_nu_are_convex_conjugates(orc, l0, l2, M):
    for x in [0.0, 1e-3, 0.05, 0.1, 2 * M * l2, 2 * M * l2 * 1.5, 0.5, 1.0, 3.0]:
        assert orc.nu(x, FIX1, l0, l2, M) == pytest.approx(conj_bf(x, FIX1, l0, l2, M), abs=1e-9)
        assert orc.nu(x, FREE, l0, l2, M) == pytest.approx(conj_bf(x, FREE, l0, l2, M), abs=1e-9)
        assert orc.nu(x, FIX0, l0, l2, M) == 0.0
        assert orc.h(x, l0, l2, M) == pytest.approx(orc.nu(x, FIX1, l0, l2, M), abs=0)


@pytest.mark.parametrize("l0,l2,M", PARAMS)
def test_z_is_argmin_of_minz(orc, l0, l2, M):
    for beta in np.linspace(0, M, 13)[1:]:
        f = lambda z: l0 * z + l2 * beta * beta / z
        r = minimize_scalar(f, bounds=(beta / M, 1.0), method="bounded", options=dict(xatol=1e-12))
        zb = min([r.x, beta / M, 1.0], key=f)
        assert orc.z(beta, FREE, l0, l2, M) == pytest.approx(zb, abs=1e-6)
    assert orc.z(0.3, FIX1, l0, l2, M) == 1.0 and orc.z(0.0, FIX0, l0, l2, M) == 0.0


# ----------------------------------------------------------------------------
# b-update, duality, ADMM
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n,p", [(30, 12), (12, 30), (20, 20)])
@pytest.mark.parametrize("rho", [1.0, 2.5])
def test_b_update_solves_normal_equations(orc, n, p, rho):
    inst = datagen.make_instance(n, p, rho=0.4, k=3, seed=5)
    o = orc.Oracle.from_instance(inst, rho=rho)
    w = np.random.default_rng(0).normal(size=p)
    b = o.b_update(w)
    A = inst.X.T @ inst.X + rho * np.eye(p)
    assert np.max(np.abs(A @ b - w)) < 1e-12 * max(1, np.max(np.abs(w)))
    assert np.allclose(o.c, inst.X.T @ inst.y, rtol=1e-13, atol=1e-14)


def test_b_update_golden_woodbury_scalar(orc):
    # tests/golden/woodbury_scalar.txt: n = 1 < p = 2 forces the Woodbury branch
    vals = {}
    for line in open(os.path.join(GOLD, "woodbury_scalar.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split("=")
            vals[k.strip()] = float(v)
    X = np.array([[1.0, 0.0]])
    o = orc.Oracle(X, np.array([1.0]), 0.01, 0.01, 10.0, rho=vals["rho"])
    b = o.b_update(np.array([1.0, 0.0]))
    assert b[0] == pytest.approx(vals["D00"], rel=1e-14)
    assert abs(b[0] - vals["D00_printed_form"]) > 0.05


def _rand_codes(rng, p, f0=0.3, f1=0.2):
    u = rng.uniform(size=p)
    return np.where(u < f0, FIX0, np.where(u < f0 + f1, FIX1, FREE)).astype(np.uint8)


@pytest.mark.parametrize("seed", range(4))
def test_weak_duality_random_points(orc, seed):
    rng = np.random.default_rng(seed)
    inst = datagen.make_instance(25, 9, rho=0.3, k=3, seed=seed, lambda0=0.02, lambda2=0.01)
    o = orc.Oracle.from_instance(inst)
    for _ in range(15):
        codes = _rand_codes(rng, 9)
        r = rng.normal(scale=rng.choice([0.05, 0.3, 1.0]), size=25)
        beta = rng.uniform(-inst.M, inst.M, 9) * (codes != FIX0)
        P = 0.5 * np.sum((inst.y - inst.X @ beta) ** 2) + sum(
            psi_bf(beta[i], codes[i], inst.lambda0, inst.lambda2, inst.M) for i in range(9))
        Dv = o.dual_value(codes, r)
        assert Dv <= P + 1e-12
        assert o.dual_bound(codes, r) <= Dv
        assert o.primal(codes, beta) == pytest.approx(P, rel=1e-8)


def _exact_dual(inst, codes, r):
    F = Fraction
    l0, l2, M = F(inst.lambda0), F(inst.lambda2), F(inst.M)
    y = [F(v) for v in inst.y]
    rr = [F(v) for v in r]
    q = -F(1, 2) * sum(a * a for a in rr) + sum(a * b for a, b in zip(y, rr))
    free_quad = l0 / l2 <= M * M
    tot = F(0)
    for j in range(inst.p):
        if codes[j] == FIX0:
            continue
        x = abs(sum(F(inst.X[i, j]) * rr[i] for i in range(inst.n)))
        hq = x * x / (4 * l2) - l0 if x <= 2 * M * l2 else M * x - l0 - l2 * M * M
        if codes[j] == FIX1:
            tot += hq
        elif free_quad:
            tot += max(hq, F(0))
        else:
            tot += max(M * x - l0 - l2 * M * M, F(0))
    return q - tot


@pytest.mark.parametrize("seed", range(3))
def test_dual_bound_is_below_exact_rational_value(orc, seed):
    rng = np.random.default_rng(10 + seed)
    inst = datagen.make_instance(7, 5, rho=0.2, k=2, seed=seed)
    o = orc.Oracle.from_instance(inst)
    for _ in range(6):
        codes = _rand_codes(rng, 5)
        r = rng.normal(scale=0.5, size=7)
        exact = _exact_dual(inst, codes, r)
        lb = o.dual_bound(codes, r)
        assert Fraction(lb) <= exact
        assert float(exact) - lb < 1e-12
        assert o.dual_value(codes, r) == pytest.approx(float(exact), abs=1e-13)


def _relax_bf(inst, codes):
    """Relaxation value by a direct minimisation of eq. relaxnode2 for tiny p, via
    coordinate-wise exact 1-D minimisation (a convex, separable-plus-smooth
    objective), independent of ADMM."""
    X, y, l0, l2, M = inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M
    p = X.shape[1]
    beta = np.zeros(p)
    for _ in range(3000):
        old = beta.copy()
        for j in range(p):
            if codes[j] == FIX0:
                beta[j] = 0.0
                continue
            rj = y - X @ beta + X[:, j] * beta[j]
            g = lambda b: 0.5 * np.sum((rj - X[:, j] * b) ** 2) + psi_bf(b, codes[j], l0, l2, M)
            r = minimize_scalar(g, bounds=(-M, M), method="bounded", options=dict(xatol=1e-13))
            beta[j] = min([r.x, 0.0, M, -M], key=g)
        if np.max(np.abs(beta - old)) < 1e-12:
            break
    P = 0.5 * np.sum((y - X @ beta) ** 2) + sum(psi_bf(beta[j], codes[j], l0, l2, M) for j in range(p))
    return P


@pytest.mark.parametrize("seed", range(3))
def test_admm_reaches_strong_duality(orc, seed):
    rng = np.random.default_rng(seed)
    inst = datagen.make_instance(30, 4, rho=0.3, k=2, seed=seed, lambda0=0.01, lambda2=0.02)
    o = orc.Oracle.from_instance(inst)
    codes = _rand_codes(rng, 4, f0=0.25, f1=0.25)
    res = o.node_admm(codes, tol=1e-11, max_iter=200000, check_every=10)
    assert res["status"] == 0
    R = _relax_bf(inst, codes)
    assert res["lb"] <= R + 1e-10
    assert res["lb"] == pytest.approx(R, abs=2e-9)
    assert res["primal"] == pytest.approx(R, abs=2e-9)


def test_relaxation_special_cases(orc):
    inst = datagen.make_instance(40, 8, rho=0.5, k=3, seed=7)
    o = orc.Oracle.from_instance(inst)
    # F0 = [p]: the relaxation is 1/2 ||y||^2
    res = o.node_admm(np.full(8, FIX0, np.uint8), tol=1e-12, max_iter=100000)
    assert res["lb"] == pytest.approx(0.5 * inst.y @ inst.y, rel=1e-9)
    # F0 u F1 = [p]: box ridge on F1 plus lambda0 |F1|
    codes = np.array([FIX1, FIX0, FIX1, FIX0, FIX0, FIX1, FIX0, FIX0], np.uint8)
    S = np.flatnonzero(codes == FIX1)
    f, _ = box_ridge(inst.X, inst.y, S, inst.lambda2, inst.M)
    res = o.node_admm(codes, tol=1e-12, max_iter=100000)
    assert res["lb"] == pytest.approx(f + inst.lambda0 * len(S), rel=1e-9)


def test_child_relaxation_not_below_parent(orc):
    rng = np.random.default_rng(4)
    inst = datagen.make_instance(30, 10, rho=0.3, k=3, seed=4)
    o = orc.Oracle.from_instance(inst)
    codes = np.zeros(10, np.uint8)
    par = o.node_admm(codes, tol=1e-10, max_iter=100000)
    for j in rng.permutation(10)[:4]:
        for fix in (FIX0, FIX1):
            c = codes.copy()
            c[j] = fix
            ch = o.node_admm(c, par["beta"], par["v"], tol=1e-10, max_iter=100000)
            assert ch["primal"] >= par["lb"] - 1e-9


# ----------------------------------------------------------------------------
# incumbent refinement
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(3))
def test_fista_and_exact_match_ridge_and_bvls(orc, seed):
    rng = np.random.default_rng(seed)
    inst = datagen.make_instance(60, 20, rho=0.4, k=4, seed=seed)
    for M in (inst.M, 0.15):
        o = orc.Oracle(inst.X, inst.y, inst.lambda0, inst.lambda2, M)
        S = np.sort(rng.choice(20, 6, replace=False))
        mask = np.zeros(20, np.uint8)
        mask[S] = 1
        fbf, bbf = box_ridge(inst.X, inst.y, S, inst.lambda2, M)
        fbf += inst.lambda0 * len(S)
        fe, be = o.exact_objective(mask)
        assert fe == pytest.approx(fbf, rel=1e-11)
        assert np.allclose(be[S], bbf, atol=1e-7)
        ff, bfi, it = o.fista(mask, np.zeros(20), tol=1e-14, max_iter=20000)
        assert ff >= fbf * (1 - 1e-12)
        assert ff == pytest.approx(fbf, rel=1e-9)
        assert np.all(bfi[mask == 0] == 0.0)
        assert o.objective(mask, bfi) == pytest.approx(ff, rel=1e-14)


def test_support_and_branch_rules(orc):
    inst = datagen.make_instance(20, 6, rho=0.1, k=2, seed=1, lambda0=0.01, lambda2=0.01, M=10.0)
    o = orc.Oracle.from_instance(inst)
    s = math.sqrt(inst.lambda0 / inst.lambda2)  # 1.0 <= M: z = min(1, |beta|/s)
    beta = np.array([0.0, 0.3 * s, 0.5 * s, 0.8 * s, 1.2 * s, 0.45 * s])
    codes = np.array([FIX1, FREE, FREE, FREE, FREE, FREE], np.uint8)
    mask, k = o.support(codes, beta)
    assert list(mask) == [1, 0, 1, 1, 1, 0] and k == 4
    assert o.branch(codes, beta) == 2          # z = 0.5 is the most fractional
    codes[2] = FIX0
    assert o.branch(codes, beta) == 5          # z = 0.45
    allint = np.array([0.0, 0.0, 2.0, 0.0, 3.0, 0.0])
    assert o.branch(np.zeros(6, np.uint8), allint) == 4   # integral: largest |beta|
    assert o.branch(np.full(6, FIX0, np.uint8), beta) == -1


# ----------------------------------------------------------------------------
# branch and bound vs enumeration
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("seed,M", [(0, None), (1, None), (2, 10.0), (3, None), (4, 0.4)])
def test_bnb_matches_enumeration(orc, seed, M):
    inst = datagen.make_instance(35, 11, rho=0.5, k=3, snr=2.0, seed=seed, lambda0=0.02,
                                 lambda2=0.01, M=M)
    o = orc.Oracle.from_instance(inst)
    res = o.bnb(tol_node=1e-7, max_iter=5000, max_iter_root=20000)
    assert res["status"] == 0
    vals = enumerate_opt(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M)
    opt, S_opt = vals[0]
    runner = vals[1][0]
    assert res["certified"] == pytest.approx(opt, rel=1e-10)
    assert res["ub"] <= opt * (1 + 1e-8)
    if (runner - opt) / opt > 1e-5:
        assert tuple(res["support"]) == S_opt
    root = res["trace"][0]
    assert root["id"] == 0 and root["lb"] <= opt * (1 + 1e-12)
    for rec in res["trace"]:
        if rec["decision"] in (0, 2):
            assert rec["ub_node"] >= opt * (1 - 1e-12)


# ----------------------------------------------------------------------------
# FISTA trajectory on a separable quadratic (closed form)
# ----------------------------------------------------------------------------

def _separable_case():
    """Two support columns that are orthogonal, with squared norms 1 and 1/4, a
    third column off the support; y has X_S^T y = (1, 0.5) exactly.  Then
    U(beta) = 1/2 ||y||^2 - c^T beta + 1/2 sum_a L_a beta_a^2 with L_a = A_a +
    2 lambda2 (A = (1, 1/4)): the gradient is L_a beta_a - c_a coordinatewise,
    and the Armijo inequality of eq. fpg_armijo at step alpha reduces to
    sum_a (alpha L_a - 1) d_a^2 <= 0 for the step d = -alpha grad (no clipping)."""
    X = np.array([[1.0, 0.0, 0.3],
                  [0.0, 0.5, 0.2],
                  [0.0, 0.0, 0.9]], order="F")
    y = np.array([1.0, 1.0, 0.7])           # X_0^T y = 1, X_1^T y = 0.5
    l0, l2, M = 0.05, 0.01, 100.0
    return X, y, l0, l2, M


def _fista_closed_form(T, mom):
    """Iterate after T steps from beta = 0: step alpha_0 = 4 / (||X_S||_F^2 + 2 lambda2)
    halved while the reduced Armijo test fails, then carried; per coordinate
    e_{t+1} = (1 - alpha L_a) (e_t + m_t (e_t - e_{t-1})) for the error
    e = beta - c / L, with the momentum m_t of the extrapolation."""
    A = np.array([1.0, 0.25])
    c = np.array([1.0, 0.5])
    l2 = 0.01
    L = A + 2 * l2
    alpha = 4.0 / (A.sum() + 2 * l2)
    g = -c                                  # gradient at the start (beta = 0)
    while np.sum((alpha * L - 1.0) * (alpha * g) ** 2) > 0.0:
        alpha *= 0.5
    q = 1.0 - alpha * L
    star = c / L
    e_prev = e = -star
    for t in range(T):
        e_new = q * (e + mom(t) * (e - e_prev))
        e_prev, e = e, e_new
    return star + e, alpha


@pytest.mark.parametrize("T", [1, 2, 3, 5, 8, 13, 21])
def test_fista_trajectory_matches_closed_form(orc, T):
    """Pins the extrapolation coefficient t/(t+3) of eq. fpg_extrapolate, the
    gradient of eq. fpg_grad, the projected step and the backtracking of
    eq. fpg_armijo with a carried step, iterate by iterate: a coefficient of
    t/(t+2), a missing 2 lambda2 or a missing 1/(2 alpha) term moves the
    iterates far beyond the tolerance."""
    X, y, l0, l2, M = _separable_case()
    o = orc.Oracle(X, y, l0, l2, M)
    mask = np.array([1, 1, 0], np.uint8)
    f, beta, it = o.fista(mask, np.zeros(3), tol=0.0, max_iter=T)
    want, alpha = _fista_closed_form(T, lambda t: t / (t + 3.0))
    assert alpha == pytest.approx(4.0 / 1.27 / 4.0, rel=1e-15)      # two halvings
    assert it == T
    assert np.max(np.abs(beta[:2] - want)) <= 1e-13
    assert beta[2] == 0.0
    if T >= 2:
        other, _ = _fista_closed_form(T, lambda t: t / (t + 2.0))
        assert np.max(np.abs(other - want)) > 1e-4


def test_fista_first_step_is_the_accepted_step_times_c(orc):
    """The same case with the Armijo test as written: the first iterate is
    alpha c (from zero, one projected gradient step), with alpha the accepted step."""
    X, y, l0, l2, M = _separable_case()
    o = orc.Oracle(X, y, l0, l2, M)
    _, beta, _ = o.fista(np.array([1, 1, 0], np.uint8), np.zeros(3), tol=0.0, max_iter=1)
    alpha = 4.0 / 1.27 / 4.0
    assert beta[:2] == pytest.approx(alpha * np.array([1.0, 0.5]), rel=1e-14)


# ----------------------------------------------------------------------------
# bounds along the path to the optimum
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("seed,M", [(0, None), (2, 10.0), (4, 0.4)])
def test_bounds_on_the_path_to_the_optimum_stay_below_opt(orc, seed, M):
    """Every node whose fixings are consistent with the optimal support S*
    (F1 within S*, F0 outside it) contains S*, so its rigorous bound, the one
    it inherits and the one it was pruned on must all be <= OPT (from
    enumeration), and they never decrease from parent to child on that path."""
    import replay
    inst = datagen.make_instance(35, 11, rho=0.5, k=3, snr=2.0, seed=seed, lambda0=0.02,
                                 lambda2=0.01, M=M)
    o = orc.Oracle.from_instance(inst)
    res = o.bnb(tol_node=1e-7, max_iter=5000, max_iter_root=20000)
    opt, S_opt = enumerate_opt(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M)[0]
    codes, _, parent = replay.node_codes(res["trace"], inst.p)
    inS = np.zeros(inst.p, bool)
    inS[list(S_opt)] = True
    lb_of = {}
    on_path = 0
    for rec in res["trace"]:
        c = codes[rec["id"]]
        lb_of[rec["id"]] = rec["lb"]
        if np.any((c == FIX1) & ~inS) or np.any((c == FIX0) & inS):
            continue
        on_path += 1
        assert rec["lb"] <= opt * (1 + 1e-12), rec
        if rec["id"] > 0:
            assert rec["lb"] >= lb_of[parent[rec["id"]]]
    assert on_path >= 1


def test_replay_of_the_oracle_own_trace_has_no_mismatch(orc):
    """The trace replayer (used against GPU traces) replaying a depth-first
    oracle trace reproduces every decision of it."""
    import replay
    inst = datagen.make_instance(35, 11, rho=0.5, k=3, snr=2.0, seed=1, lambda0=0.02, lambda2=0.01)
    o = orc.Oracle.from_instance(inst)
    kw = dict(tol_node=1e-7, max_iter=5000, max_iter_root=20000, check_every=10)
    res = o.bnb(**kw, eps_prune=2e-7)
    out = replay.replay(o, res["trace"], eps_prune=2e-7, **kw)
    assert out["mismatch"] == []
    assert out["solved"] == res["nodes_solved"]
    assert out["prune_cmp"] + out["prune_band"] == out["solved"]
    assert out["branch_cmp"] > 0


@pytest.mark.parametrize("n,p", [(40, 25), (25, 40)])
def test_factored_constructor_matches_the_plain_one(orc, n, p):
    """The oracle with its once-per-tree factor taken from numpy (used for the
    large instances) gives the same b-update and node solves as the oracle that
    forms the factor itself, in both forms (D for n >= p, the Cholesky factor of
    X X^T + rho I for n < p)."""
    inst = datagen.make_instance(n, p, rho=0.4, k=3, seed=7)
    a = orc.Oracle.from_instance(inst, rho=0.7)
    b = orc.Oracle.from_instance(inst, rho=0.7, factor="numpy")
    w = np.random.default_rng(1).normal(size=p)
    assert np.max(np.abs(a.b_update(w) - b.b_update(w))) <= 1e-12 * np.max(np.abs(w))
    codes = np.zeros(p, np.uint8)
    codes[:3] = [FIX0, FIX1, FIX0]
    ra = a.node_admm(codes, tol=1e-8, max_iter=20000)
    rb = b.node_admm(codes, tol=1e-8, max_iter=20000)
    assert ra["status"] == rb["status"] == 0
    assert abs(ra["lb"] - rb["lb"]) <= 1e-9 * abs(ra["primal"])


# ----------------------------------------------------------------------------
# matching-pursuit root heuristic (Sec. 3.5, App. A.2)
# ----------------------------------------------------------------------------

def _F(X, y, l0, l2, beta, mask):
    """F(S, beta) = 1/2 ||y - X beta||^2 + l2 ||beta||^2 + l0 |S|, written out."""
    r = y - X @ beta
    return 0.5 * float(r @ r) + l2 * float(beta @ beta) + l0 * int(mask.sum())


def _mp_state(rng, n, p, M):
    X = rng.standard_normal((n, p))
    X /= np.linalg.norm(X, axis=0)
    y = rng.standard_normal(n)
    y /= np.linalg.norm(y)
    mask = (rng.random(p) < 0.4).astype(np.uint8)
    beta = np.where(mask == 1, rng.uniform(-M, M, p), 0.0)
    return X, y, mask, beta


@pytest.mark.parametrize("seed,M", [(0, 10.0), (1, 0.3), (2, 0.05)])
def test_mp_deltas_match_one_coordinate_brute_force(orc, seed, M):
    """Forward Delta_j = min over |b| <= M of F(S + j, beta + b e_j) - F(S, beta)
    (grid, then a bounded scalar search); backward Delta_j = F(S - j, beta with
    beta_j = 0) - F(S, beta), evaluated directly."""
    rng = np.random.default_rng(seed)
    n, p, l0, l2 = 30, 9, 0.01, 0.02
    X, y, mask, beta = _mp_state(rng, n, p, M)
    o = orc.Oracle(X, y, l0, l2, M)
    r = y - X @ beta
    delta, bnew = o.mp_deltas(mask, beta, r)
    F0 = _F(X, y, l0, l2, beta, mask)
    for j in range(p):
        if mask[j]:
            b2, m2 = beta.copy(), mask.copy()
            b2[j], m2[j] = 0.0, 0
            assert abs(delta[j] - (_F(X, y, l0, l2, b2, m2) - F0)) <= 1e-12
            assert bnew[j] == 0.0
            continue
        m2 = mask.copy()
        m2[j] = 1

        def g(b):
            b2 = beta.copy()
            b2[j] = b
            return _F(X, y, l0, l2, b2, m2) - F0

        grid = np.linspace(-M, M, 4001)
        vals = np.array([g(b) for b in grid])
        k = int(np.argmin(vals))
        lo, hi = grid[max(k - 1, 0)], grid[min(k + 1, len(grid) - 1)]
        res = minimize_scalar(g, bounds=(lo, hi), method="bounded", options=dict(xatol=1e-12))
        best = min(res.fun, vals[k])
        assert abs(delta[j] - best) <= 1e-10
        assert delta[j] <= best + 1e-13
        assert abs(bnew[j] - (res.x if res.fun <= vals[k] else grid[k])) <= 1e-5


@pytest.mark.parametrize("seed,M", [(0, 10.0), (3, 0.2), (5, 1.0)])
def test_mp_moves_lower_F_by_their_delta_and_end_locally_optimal(orc, seed, M):
    """Replaying the moves: each lowers F by exactly the Delta of its state (and
    is the smallest of its kind, ties to the smallest index); at exit no single
    addition or removal lowers F."""
    rng = np.random.default_rng(seed)
    n, p, l0, l2 = 40, 14, 0.005, 0.01
    X, y, _, _ = _mp_state(rng, n, p, M)
    y = X[:, [1, 6, 11]] @ np.array([0.8, -0.5, 0.6]) + 0.3 * y
    o = orc.Oracle(X, y, l0, l2, M)
    mask_f, beta_f, moves = o.matching_pursuit()
    assert moves and moves[0] > 0
    mask = np.zeros(p, np.uint8)
    beta = np.zeros(p)
    F = _F(X, y, l0, l2, beta, mask)
    for mv in moves:
        j = abs(mv) - 1
        delta, bnew = o.mp_deltas(mask, beta, y - X @ beta)
        cand = np.flatnonzero(mask == (0 if mv > 0 else 1))
        assert delta[j] < 0 and j == cand[np.argmin(delta[cand])]
        if mv > 0:
            beta[j], mask[j] = bnew[j], 1
        else:
            beta[j], mask[j] = 0.0, 0
        F_new = _F(X, y, l0, l2, beta, mask)
        assert abs((F_new - F) - delta[j]) <= 1e-12
        F = F_new
    assert np.array_equal(mask, mask_f) and np.allclose(beta, beta_f, rtol=0, atol=1e-14)
    delta, _ = o.mp_deltas(mask, beta, y - X @ beta)
    assert np.all(delta >= 0.0)


@pytest.mark.parametrize("seed,M", [(0, 10.0), (1, 0.25)])
def test_mp_reaches_the_global_optimum_on_orthonormal_designs(orc, seed, M):
    """With orthonormal columns F separates over coordinates, so the frozen
    one-coordinate moves are exact and the heuristic must end at the optimum
    found by enumerating every support."""
    rng = np.random.default_rng(seed)
    n, p, l0, l2 = 30, 10, 0.01, 0.02
    Q, _ = np.linalg.qr(rng.standard_normal((n, p)))
    y = Q @ rng.uniform(-0.6, 0.6, p) + 0.05 * rng.standard_normal(n)
    o = orc.Oracle(np.asfortranarray(Q), y, l0, l2, M)
    mask, beta, moves = o.matching_pursuit()
    assert all(m > 0 for m in moves)
    vals = enumerate_opt(Q, y, l0, l2, M)
    f_opt, S_opt = vals[0]
    assert vals[1][0] - f_opt > 1e-9
    assert tuple(np.flatnonzero(mask)) == S_opt
    assert abs(_F(Q, y, l0, l2, beta, mask) - f_opt) <= 1e-12
