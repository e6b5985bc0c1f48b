"""Parity of the HIP library (through its C ABI) with the FP64 CPU oracle on the
same seeded inputs.  Bars: FP64 iterates within 1e-11 relative, equal sweep
counts, bit-exact rounding/branching and BnB traces in FP64 DFS; FP32 node
bounds within 1e-5 relative; certified objectives within 1e-8 relative and the
same optimal support."""
import numpy as np
import pytest

from paper_2602_04551_amd import datagen

pytestmark = pytest.mark.gpu
FREE, FIX0, FIX1 = 0, 1, 2


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def ctx_for(inst, precision, rho=1.0):
    from paper_2602_04551_amd.binding import Context
    c = Context(0)
    c.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, rho=rho, precision=precision)
    return c


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


def random_nodes(p, K, seed, base_beta, base_v, nfix=(1, 6)):
    rng = np.random.default_rng(seed)
    codes = np.zeros((K, p), np.uint8)
    for k in range(K):
        f = rng.integers(nfix[0], nfix[1] + 1)
        idx = rng.choice(p, size=min(f, p), replace=False)
        codes[k, idx] = rng.choice([FIX0, FIX1], size=len(idx))
    beta = np.tile(base_beta, (K, 1)) + rng.normal(scale=1e-3, size=(K, p))
    v = np.tile(base_v, (K, 1)) + rng.normal(scale=1e-3, size=(K, p))
    return codes, beta, v


INSTANCES = {
    "C1": lambda: datagen.config_instance("C1", seed=0),
    "wide": lambda: datagen.make_instance(70, 150, rho=0.4, k=4, seed=3, lambda0=0.01, lambda2=0.01),
    "ragged": lambda: datagen.make_instance(97, 45, rho=0.2, k=3, seed=4, lambda0=0.02, lambda2=0.01, M=10.0),
}


@pytest.fixture(scope="module")
def cases(orc):
    out = {}
    for name, mk in INSTANCES.items():
        inst = mk()
        o = orc.Oracle.from_instance(inst)
        root = o.node_admm(None, tol=1e-7, max_iter=20000)
        out[name] = (inst, o, root)
    return out


@pytest.mark.parametrize("name", list(INSTANCES))
def test_sweeps_fp64_match_oracle(torch_cuda, cases, name):
    inst, o, root = cases[name]
    K = 37
    codes, beta0, v0 = random_nodes(inst.p, K, 1, root["beta"], root["v"])
    ctx = ctx_for(inst, "fp64")
    for S in (1, 25):
        gb, gv, gbb = ctx.admm_sweeps(codes, beta0, v0, S)
        gb, gv, gbb = gb.cpu().numpy(), gv.cpu().numpy(), gbb.cpu().numpy()
        for k in range(K):
            b = beta0[k].copy()
            b[codes[k] == FIX0] = 0.0
            v = v0[k].copy()
            for _ in range(S):
                b, v, bb = o.sweep(codes[k], b, v)
            assert rel(gb[k], b) < 1e-11, (S, k)
            assert rel(gv[k], v) < 1e-11, (S, k)
            assert rel(gbb[k], bb) < 1e-11, (S, k)


@pytest.mark.parametrize("rho", [0.7, 2.0, 0.3])
def test_sweeps_and_node_solve_other_rho(torch_cuda, orc, rho):
    """rho other than 1: a power of two (the update multiplies by 1/rho, which is
    exact) and two that are not (it divides); sweeps and FP64 node solves match
    the oracle run with the same rho, sweep counts included."""
    inst = INSTANCES["wide"]()
    o = orc.Oracle.from_instance(inst, rho=rho)
    root = o.node_admm(None, tol=1e-7, max_iter=20000)
    K = 24
    codes, beta0, v0 = random_nodes(inst.p, K, 21, root["beta"], root["v"])
    ctx = ctx_for(inst, "fp64", rho=rho)
    gb, gv, gbb = ctx.admm_sweeps(codes, beta0, v0, 9)
    gb, gv, gbb = gb.cpu().numpy(), gv.cpu().numpy(), gbb.cpu().numpy()
    for k in range(K):
        b = beta0[k].copy()
        b[codes[k] == FIX0] = 0.0
        v = v0[k].copy()
        for _ in range(9):
            b, v, bb = o.sweep(codes[k], b, v)
        assert rel(gb[k], b) < 1e-11 and rel(gv[k], v) < 1e-11 and rel(gbb[k], bb) < 1e-11, k
    res = ctx.solve_node_batch(codes, beta0, v0, tol_node=1e-7, max_iter=3000, check_every=10)
    it, lb = res["iters"].cpu().numpy(), res["lb"].cpu().numpy()
    for k in range(K):
        ref = o.node_admm(codes[k], beta0[k], v0[k], tol=1e-7, max_iter=3000, check_every=10)
        assert it[k] == ref["iters"], k
        assert abs(lb[k] - ref["lb"]) <= 1e-10 * abs(ref["primal"]), k


@pytest.mark.parametrize("shape", list(range(18)))
def test_every_tile_shape_matches_oracle(torch_cuda, cases, shape):
    """Every shape of the contraction over p (12-17: LDS or register tiles with
    the range cut into slices) and of the contraction over n."""
    inst, o, root = cases["ragged"]
    K = 100
    codes, beta0, v0 = random_nodes(inst.p, K, 11, root["beta"], root["v"])
    ctx = ctx_for(inst, "fp64")
    ctx.set_tiles(shape, 11 - shape if shape < 12 else 0)
    gb, gv, gbb = ctx.admm_sweeps(codes, beta0, v0, 7)
    gb, gbb = gb.cpu().numpy(), gbb.cpu().numpy()
    for k in range(K):
        b = beta0[k].copy()
        b[codes[k] == FIX0] = 0.0
        v = v0[k].copy()
        for _ in range(7):
            b, v, bb = o.sweep(codes[k], b, v)
        assert rel(gb[k], b) < 1e-11 and rel(gbb[k], bb) < 1e-11


@pytest.mark.parametrize("shape", [9, 10, 11, 12, 13])
def test_lds_tiles_fp32_and_anchored_match(torch_cuda, cases, shape):
    """The LDS-staged tiles in FP32 mode (plain and anchored sweeps, with the gap
    estimate's epilogue) give the same node solves as the register tiles, to
    FP32 rounding of the summation order."""
    _fp32_shape_matches(cases, shape)


@pytest.mark.parametrize("shape", [6, 7, 8])
def test_large_register_tiles_fp32_and_anchored_match(torch_cuda, cases, shape):
    """The 64 x 32, 32 x 64 and 64 x 64 register tiles in FP32 mode (both
    contractions, plain and anchored sweeps) give the same node solves as the
    32 x 32 register tile, to FP32 rounding of the summation order."""
    _fp32_shape_matches(cases, shape)


def _fp32_shape_matches(cases, shape):
    inst, o, root = cases["wide"]
    K = 128
    codes, beta0, v0 = random_nodes(inst.p, K, 13, root["beta"], root["v"])
    ref = ctx_for(inst, "fp32")
    ref.set_tiles(1, 1)
    r0 = ref.solve_node_batch(codes, beta0, v0, tol_node=1e-8, max_iter=3000, check_every=10)
    ctx = ctx_for(inst, "fp32")
    ctx.set_tiles(shape, min(shape, 11))
    r1 = ctx.solve_node_batch(codes, beta0, v0, tol_node=1e-8, max_iter=3000, check_every=10)
    lb0, lb1 = r0["lb"].cpu().numpy(), r1["lb"].cpu().numpy()
    pr = r0["primal"].cpu().numpy()
    assert (r1["status"].cpu().numpy() == 0).all()
    assert np.max(np.abs(lb0 - lb1) / np.abs(pr)) < 1e-7


@pytest.mark.parametrize("shape", [1, 2])
def test_bf16_lds_tiles_match_the_register_tile(torch_cuda, cases, shape):
    """BF16 split form: the LDS-staged tiles (64 x 64, 128 x 128; the FP32 node
    operand split into hi / lo as it is staged) for both contractions give the
    same node solves as the register tiles, to FP32 rounding of the summation
    order, and agree with the oracle's bounds."""
    inst, o, root = cases["wide"]
    K = 128
    codes, beta0, v0 = random_nodes(inst.p, K, 14, root["beta"], root["v"])
    ref = ctx_for(inst, "bf16")
    ref.set_tiles(0, 0)
    r0 = ref.solve_node_batch(codes, beta0, v0, tol_node=1e-8, max_iter=3000, check_every=10)
    ctx = ctx_for(inst, "bf16")
    ctx.set_tiles(shape, shape)
    r1 = ctx.solve_node_batch(codes, beta0, v0, tol_node=1e-8, max_iter=3000, check_every=10)
    lb0, lb1 = r0["lb"].cpu().numpy(), r1["lb"].cpu().numpy()
    pr = r0["primal"].cpu().numpy()
    assert (r1["status"].cpu().numpy() == 0).all()
    assert np.max(np.abs(lb0 - lb1) / np.abs(pr)) < 1e-7
    for k in range(0, K, 16):
        ref_k = o.node_admm(codes[k], beta0[k], v0[k], tol=1e-8, max_iter=3000, check_every=10)
        assert abs(lb1[k] - ref_k["lb"]) <= 1e-7 * abs(ref_k["primal"])


@pytest.mark.parametrize("shape", [1, 2])
def test_fp8_lds_tiles_match_the_register_tile(torch_cuda, cases, shape):
    """FP8 storage: the LDS-staged contraction over n (64 x 64, 128 x 128) gives
    the same anchored node solves as the register tile, to FP32 rounding of the
    summation order, and both agree with the oracle's bounds."""
    inst, o, root = cases["wide"]
    K = 128
    codes, beta0, v0 = random_nodes(inst.p, K, 13, root["beta"], root["v"])
    ref = ctx_for(inst, "fp8")
    ref.set_tiles(0, 0)
    r0 = ref.solve_node_batch(codes, beta0, v0, tol_node=1e-8, max_iter=3000, check_every=10)
    ctx = ctx_for(inst, "fp8")
    ctx.set_tiles(0, shape)
    r1 = ctx.solve_node_batch(codes, beta0, v0, tol_node=1e-8, max_iter=3000, check_every=10)
    lb0, lb1 = r0["lb"].cpu().numpy(), r1["lb"].cpu().numpy()
    pr = r0["primal"].cpu().numpy()
    assert (r1["status"].cpu().numpy() == 0).all()
    assert np.max(np.abs(lb0 - lb1) / np.abs(pr)) < 1e-7
    for k in range(0, K, 16):
        ref_k = o.node_admm(codes[k], beta0[k], v0[k], tol=1e-8, max_iter=3000, check_every=10)
        assert abs(lb1[k] - ref_k["lb"]) <= 1e-7 * abs(ref_k["primal"])


SLICED = [("bf16", 13), ("bf16", 15), ("bf16", 17), ("fp8", 13), ("fp8", 15), ("fp8", 17), ("fp32", 13),
          ("fp32", 17)]


@pytest.mark.parametrize("shape_name", ["wide", "long"])
@pytest.mark.parametrize("precision,xw", SLICED)
def test_sliced_contraction_over_p_matches_unsliced(torch_cuda, cases, orc, precision, xw, shape_name):
    """The contraction over p cut into 4 or 8 slices (partial products added in
    slice order; register or 128 x 128 LDS-staged tiles) gives the same node
    solves as the unsliced register tile, to FP32 rounding of the summation
    order.  (The FP64 anchors take the fixed shape too; the LDS tiles take 128
    nodes, so the batch is 128.)  "long" has p = 300: its padded range of 384 is
    12 chunks of 32, so 8 slices are uneven (1 or 2 chunks each)."""
    if shape_name == "wide":
        inst, o, root = cases["wide"]
    else:
        inst = datagen.make_instance(60, 300, rho=0.3, k=4, seed=9, lambda0=0.01, lambda2=0.01)
        root = orc.Oracle.from_instance(inst).node_admm(None, tol=1e-7, max_iter=20000)
    K = 128
    codes, beta0, v0 = random_nodes(inst.p, K, 17, root["beta"], root["v"])
    ref = ctx_for(inst, precision)
    ref.set_tiles(0, 0)
    r0 = ref.solve_node_batch(codes, beta0, v0, tol_node=1e-8, max_iter=3000, check_every=10)
    ctx = ctx_for(inst, precision)
    ctx.set_tiles(xw, 0)
    r1 = ctx.solve_node_batch(codes, beta0, v0, tol_node=1e-8, max_iter=3000, check_every=10)
    lb0, lb1 = r0["lb"].cpu().numpy(), r1["lb"].cpu().numpy()
    pr = r0["primal"].cpu().numpy()
    assert (r1["status"].cpu().numpy() == 0).all()
    assert np.max(np.abs(lb0 - lb1) / np.abs(pr)) < 1e-7


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16", "fp8"])
def test_live_bucket_narrower_than_the_batch_with_sliced_tiles(torch_cuda, precision):
    """Few rows and a long p: the tuner takes sliced contractions over p.  Once
    fewer than half of a 64-node batch is live, the launches cover a 32-column
    bucket whose columns name slots up to 63; each slice's partial products are
    kept per slot, so the node results equal those of a fixed unsliced shape
    (which always covers the whole batch)."""
    inst = datagen.make_instance(200, 4000, rho=0.3, k=5, seed=5, lambda0=0.01, lambda2=0.01)
    K = 64
    zero = np.zeros(inst.p)
    codes, beta0, v0 = random_nodes(inst.p, K, 31, zero, zero, nfix=(1, 40))
    ref = ctx_for(inst, precision)
    ref.set_tiles(0, 0)
    r0 = ref.solve_node_batch(codes, beta0, v0, tol_node=1e-6, max_iter=3000, check_every=10)
    ctx = ctx_for(inst, precision)
    r1 = ctx.solve_node_batch(codes, beta0, v0, tol_node=1e-6, max_iter=3000, check_every=10)
    it0, it1 = r0["iters"].cpu().numpy(), r1["iters"].cpu().numpy()
    st0, st1 = r0["status"].cpu().numpy(), r1["status"].cpu().numpy()
    lb0, lb1 = r0["lb"].cpu().numpy(), r1["lb"].cpu().numpy()
    pr = r0["primal"].cpu().numpy()
    conv = st0 == 0
    assert conv.sum() >= 48
    # the batch thins out: the last half of the nodes run on after the first half converged
    assert np.sort(it0)[31] < it0.max()
    if precision == "fp64":
        assert (st0 == st1).all() and (it0 == it1).all()
        assert np.max(np.abs(lb0 - lb1) / np.abs(pr)) < 1e-10
    else:
        both = conv & (st1 == 0)
        assert both.sum() >= conv.sum() - 2
        assert np.max(np.abs(lb0 - lb1)[both] / np.abs(pr[both])) < 1e-6


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_size_tuner_and_bnb_with_tuned_K(torch_cuda, orc, precision):
    """The batch axis of the autotuner: one positive rate per candidate K, the
    chosen K the smallest within the fraction of the best rate, and a best-first
    BnB with K = 0 (tuned) certifying the oracle's optimum."""
    from paper_2602_04551_amd.binding import L0L2Error
    inst = datagen.config_instance("C1", seed=0)
    ctx = ctx_for(inst, precision)
    K, rates = ctx.tune_batch_size(k_max=256, frac=0.9)
    assert list(rates) == [32, 64, 128, 256] and all(r > 0 for r in rates.values())
    best = max(rates.values())
    assert rates[K] >= 0.9 * best and all(rates[k] < 0.9 * best for k in rates if k < K)
    r = ctx.bnb_solve(K=0, policy="best", tol_node=1e-6, max_iter=2000)
    o = orc.Oracle.from_instance(inst)
    ref = o.bnb(tol_node=1e-6, max_iter=2000)
    assert r["status"] == 0
    assert abs(r["certified"] - ref["certified"]) <= 1e-8 * abs(ref["certified"])
    assert sorted(r["support"].tolist()) == sorted(np.flatnonzero(ref["mask"]).tolist())
    with pytest.raises(L0L2Error):
        ctx.tune_batch_size(k_max=16)


@pytest.mark.parametrize("precision,check_every,tol", [("fp32", 10, 1e-7), ("fp32", 7, 1e-7),
                                                       ("bf16", 10, 1e-6), ("bf16", 7, 1e-6)])
def test_gram_form_matches_folded_form_and_oracle(torch_cuda, cases, precision, check_every, tol):
    """FP32 and BF16 modes, b-update through G = Xh^T Xh (one contraction per
    sweep, W in two alternating buffers; BF16: G as a BF16 pair) against the
    folded form (two contractions): every node converges to the same bounds, and
    to the oracle's.  An odd block length leaves W in the second buffer at block
    ends (copied back)."""
    inst, o, root = cases["C1"]
    K = 96
    codes, beta0, v0 = random_nodes(inst.p, K, 23, root["beta"], root["v"])
    res = {}
    for form in ("folded", "gram"):
        ctx = ctx_for(inst, precision)
        ctx.set_bupdate_form(form)
        res[form] = ctx.solve_node_batch(codes, beta0, v0, tol_node=1e-8, max_iter=3000, check_every=check_every)
    lb0, lb1 = res["folded"]["lb"].cpu().numpy(), res["gram"]["lb"].cpu().numpy()
    pr = res["folded"]["primal"].cpu().numpy()
    assert (res["gram"]["status"].cpu().numpy() == 0).all()
    assert np.max(np.abs(lb0 - lb1) / np.abs(pr)) < tol
    for k in range(0, K, 12):
        ref = o.node_admm(codes[k], beta0[k], v0[k], tol=1e-8, max_iter=3000, check_every=check_every)
        assert abs(lb1[k] - ref["lb"]) <= tol * abs(ref["primal"]), k


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("shape", ["wide", "tall"])
def test_gram_form_with_unequal_padded_extents(torch_cuda, cases, orc, precision, shape):
    """The Gram form where the padded p differs from the padded n: forced on a
    wide design (n = 70, p = 150: 128 against 256 padded, where the default is
    the folded operand) and by default on a tall one (n = 300, p = 100: 384
    against 128).  The tile shapes are timed on the folded operands, whose
    contraction over n has another length than the Gram form's over p."""
    if shape == "wide":
        inst, o, root = cases["wide"]
    else:
        inst = datagen.make_instance(300, 100, rho=0.3, k=5, seed=6, lambda0=0.01, lambda2=0.01)
        o = orc.Oracle.from_instance(inst)
        root = o.node_admm(None, tol=1e-7, max_iter=20000)
    tol = 1e-7 if precision == "fp32" else 1e-6
    K = 45
    codes, beta0, v0 = random_nodes(inst.p, K, 41, root["beta"], root["v"])
    res = {}
    for form in ("folded", "gram"):
        ctx = ctx_for(inst, precision)
        ctx.set_bupdate_form(form)
        r = ctx.solve_node_batch(codes, beta0, v0, tol_node=1e-8, max_iter=4000, check_every=7)
        res[form] = {k: v.cpu().numpy() for k, v in r.items()}
    f, g = res["folded"], res["gram"]
    assert np.all(g["lb"] <= g["primal"])
    conv = (f["status"] == 0) & (g["status"] == 0)
    assert conv.sum() >= K - 2
    assert np.max(np.abs(f["lb"] - g["lb"])[conv] / np.abs(f["primal"][conv])) < tol
    for k in range(0, K, 9):
        if not conv[k]:
            continue
        ref = o.node_admm(codes[k], beta0[k], v0[k], tol=1e-8, max_iter=4000, check_every=7)
        assert abs(g["lb"][k] - ref["lb"]) <= tol * abs(ref["primal"]), k


def test_fixed_shape_that_does_not_fit_the_batch_is_rejected(torch_cuda, cases):
    """Shape 7 tiles 64 nodes; a batch padded to 32 nodes cannot use it."""
    from paper_2602_04551_amd.binding import L0L2Error
    inst, o, root = cases["ragged"]
    codes, beta0, v0 = random_nodes(inst.p, 20, 12, root["beta"], root["v"])
    ctx = ctx_for(inst, "fp64")
    ctx.set_tiles(7, 1)
    with pytest.raises(L0L2Error):
        ctx.admm_sweeps(codes, beta0, v0, 2)
    ctx.set_tiles(-1, -1)
    ctx.admm_sweeps(codes, beta0, v0, 2)


@pytest.mark.parametrize("precision,tol", [("fp32", 2e-5), ("bf16", 5e-4)])
def test_sweeps_reduced_precision_close_to_oracle(torch_cuda, cases, precision, tol):
    """FP32 sweeps, and the BF16 split form (two BF16 terms per operand, FP32
    accumulation), stay within their operator accuracy of the FP64 oracle."""
    inst, o, root = cases["C1"]
    K = 33
    codes, beta0, v0 = random_nodes(inst.p, K, 2, root["beta"], root["v"])
    ctx = ctx_for(inst, precision)
    gb, gv, _ = ctx.admm_sweeps(codes, beta0, v0, 5)
    gb, gv = gb.cpu().numpy(), gv.cpu().numpy()
    for k in range(K):
        b = beta0[k].astype(np.float32).astype(np.float64)
        b[codes[k] == FIX0] = 0.0
        v = v0[k].astype(np.float32).astype(np.float64)
        for _ in range(5):
            b, v, _ = o.sweep(codes[k], b, v)
        assert rel(gb[k], b) < tol
        assert rel(gv[k], v) < tol


@pytest.mark.parametrize("name", list(INSTANCES))
def test_dual_bound_fp64_matches_oracle(torch_cuda, cases, name):
    inst, o, root = cases[name]
    K = 40
    codes, beta0, v0 = random_nodes(inst.p, K, 3, root["beta"], root["v"])
    bvec = np.stack([o.sweep(codes[k], beta0[k] * (codes[k] != FIX0), v0[k])[2] for k in range(K)])
    ctx = ctx_for(inst, "fp64")
    lb = ctx.dual_bound(codes, bvec).cpu().numpy()
    for k in range(K):
        r = inst.y - inst.X @ bvec[k]
        ref = o.dual_bound(codes[k], r)
        assert abs(lb[k] - ref) <= 1e-12 * max(1.0, abs(ref))
        assert lb[k] <= o.dual_value(codes[k], r) + 1e-15


@pytest.mark.parametrize("name", list(INSTANCES))
def test_node_solve_fp64_matches_oracle(torch_cuda, cases, name):
    inst, o, root = cases[name]
    K = 45
    codes, beta0, v0 = random_nodes(inst.p, K, 4, root["beta"], root["v"])
    ctx = ctx_for(inst, "fp64")
    res = ctx.solve_node_batch(codes, beta0, v0, tol_node=1e-7, max_iter=3000, check_every=10)
    lb, pr = res["lb"].cpu().numpy(), res["primal"].cpu().numpy()
    it, stt = res["iters"].cpu().numpy(), res["status"].cpu().numpy()
    gb = res["beta"].cpu().numpy()
    for k in range(K):
        ref = o.node_admm(codes[k], beta0[k], v0[k], tol=1e-7, max_iter=3000, check_every=10)
        assert it[k] == ref["iters"] and stt[k] == ref["status"], k
        assert abs(lb[k] - ref["lb"]) <= 1e-10 * abs(ref["primal"])
        assert abs(pr[k] - ref["primal"]) <= 1e-10 * abs(ref["primal"])
        assert rel(gb[k], ref["beta"]) < 1e-9


@pytest.mark.parametrize("name,precision", [("C1", "fp32"), ("wide", "fp32"), ("C1", "bf16"),
                                            ("wide", "bf16"), ("C1", "fp8"), ("wide", "fp8")])
def test_node_solve_mixed_bounds_within_1e5(torch_cuda, cases, name, precision):
    """Mixed paths: FP32 (or BF16 split) sweeps, then anchored sweeps on the FP64
    state; FP8 storage anchored from the start.  Every node reaches the 1e-6 gap
    and its FP64 bound is within 1e-5 of the oracle's."""
    inst, o, root = cases[name]
    K = 40
    codes, beta0, v0 = random_nodes(inst.p, K, 5, root["beta"], root["v"])
    ctx = ctx_for(inst, precision)
    ctx.profile_enable(True)
    res = ctx.solve_node_batch(codes, beta0, v0, tol_node=1e-6, max_iter=4000, check_every=10)
    n32 = ctx.profile_query("admm_xtu." + {"fp32": "f32", "bf16": "bf16", "fp8": "fp8"}[precision])[0]
    assert n32 > 0
    lb, stt = res["lb"].cpu().numpy(), res["status"].cpu().numpy()
    for k in range(K):
        ref = o.node_admm(codes[k], beta0[k], v0[k], tol=1e-6, max_iter=4000, check_every=10)
        assert stt[k] == 0
        assert abs(lb[k] - ref["lb"]) <= 1e-5 * abs(ref["primal"])
        assert lb[k] <= ref["primal"] + 1e-12


@pytest.mark.parametrize("name,precision", [("C1", "fp32"), ("wide", "fp32"), ("C1", "bf16"), ("wide", "bf16"),
                                            ("C1", "fp8"), ("wide", "fp8")])
def test_reduced_modes_reach_fp64_tolerances(torch_cuda, cases, name, precision):
    """FP32, BF16 and FP8 modes below their own rounding floors: the anchored
    sweeps on the FP64 state multiply only the movement since the block's FP64
    anchor (in FP32, in the BF16 split form, or with the FP8 codes), so a 1e-9
    gap is reached and the FP64 bound agrees with the oracle's to 1e-8 of the
    primal value."""
    inst, o, root = cases[name]
    K = 24
    codes, beta0, v0 = random_nodes(inst.p, K, 8, root["beta"], root["v"])
    ctx = ctx_for(inst, precision)
    ctx.profile_enable(True)
    res = ctx.solve_node_batch(codes, beta0, v0, tol_node=1e-9, max_iter=6000, check_every=10)
    assert ctx.profile_query("anchor.f64")[0] > 0
    assert ctx.profile_query("admm_xtu.f64")[0] == 0
    lb, stt = res["lb"].cpu().numpy(), res["status"].cpu().numpy()
    for k in range(K):
        ref = o.node_admm(codes[k], beta0[k], v0[k], tol=1e-9, max_iter=6000, check_every=10)
        assert stt[k] == 0
        assert abs(lb[k] - ref["lb"]) <= 1e-8 * abs(ref["primal"])
        assert lb[k] <= ref["primal"] + 1e-12


@pytest.mark.parametrize("name", list(INSTANCES))
def test_round_branch_bit_exact(torch_cuda, cases, name):
    inst, o, root = cases[name]
    K = 50
    codes, beta0, v0 = random_nodes(inst.p, K, 6, root["beta"], root["v"])
    beta0 = beta0 * (codes != FIX0)
    beta0[3] = 0.0           # all-zero iterate: every free score is 0
    codes[4] = FIX0          # no free coordinate
    ctx = ctx_for(inst, "fp64")
    out = ctx.round_branch(codes, beta0)
    sup = out["support"].cpu().numpy()
    for k in range(K):
        mask, cnt = o.support(codes[k], beta0[k])
        assert np.array_equal(sup[k], mask) and out["support_size"][k].item() == cnt
        j = o.branch(codes[k], beta0[k])
        assert out["branch_j"][k].item() == j
    assert out["branch_j"][4].item() == -1


@pytest.mark.parametrize("name", ["C1", "ragged"])
def test_refine_incumbent_matches_oracle(torch_cuda, cases, name):
    inst, o, root = cases[name]
    K = 24
    rng = np.random.default_rng(7)
    sup = np.zeros((K, inst.p), np.uint8)
    for k in range(K):
        sup[k, rng.choice(inst.p, size=rng.integers(0, 9), replace=False)] = 1
    start = np.tile(root["beta"], (K, 1))
    ctx = ctx_for(inst, "fp64")
    obj, beta, _ = ctx.refine_incumbent(sup, start, tol=1e-12, max_iter=1000)
    obj32, _, _ = ctx_for(inst, "fp32").refine_incumbent(sup, start, tol=1e-12, max_iter=1000)
    assert np.all(np.abs(obj32.cpu().numpy() - obj.cpu().numpy()) <= 1e-8 * obj.cpu().numpy())
    obj, beta = obj.cpu().numpy(), beta.cpu().numpy()
    u = 2.0 ** -53
    for k in range(K):
        f, b, _ = o.fista(sup[k], start[k], tol=1e-12, max_iter=1000)
        assert abs(obj[k] - f) <= 1e-10 * f
        fe, bstar = o.exact_objective(sup[k])
        g, _ = ctx.exact_objective(sup[k])
        assert abs(g - fe) <= 1e-12 * fe
        # Iterates: U restricted to S is strongly convex with modulus mu = the
        # smallest eigenvalue of X_S^T X_S + 2 lambda2 I, and the minimiser b* over
        # the box satisfies U(b) - U(b*) >= mu/2 ||b - b*||^2 for every feasible b.
        # F is evaluated by the oracle in FP64; each evaluation is off by at most
        # e_F = (n + |S| + 4) u (||y|| + ||X_S||_F ||b||)^2 (n squared residuals,
        # each an |S|-term inner product), and the exact re-solve's point bstar is
        # itself a feasible point with F(bstar) <= F* + 2 e_F.  So every feasible b
        # lies within r(b) = sqrt(2 (F(b) - F(bstar) + 2 e_F) / mu) of b*, bstar
        # within sqrt(4 e_F / mu) of it, and two points within the sum of radii.
        S = np.flatnonzero(sup[k])
        if len(S) == 0:
            assert np.all(beta[k] == 0.0)
            continue
        XS = inst.X[:, S]
        H = XS.T @ XS + 2 * inst.lambda2 * np.eye(len(S))
        mu = float(np.linalg.eigvalsh(H)[0])
        xs_f = float(np.linalg.norm(XS))
        scale = max(np.linalg.norm(beta[k][S]), np.linalg.norm(b[S]), np.linalg.norm(bstar[S]))
        e_F = (inst.n + len(S) + 4) * u * (np.linalg.norm(inst.y) + xs_f * scale) ** 2

        def radius(v):
            return np.sqrt(2 * (max(o.objective(sup[k], v) - fe, 0.0) + 2 * e_F) / mu)

        r_star = np.sqrt(4 * e_F / mu)
        assert np.linalg.norm(beta[k] - bstar) <= radius(beta[k]) + r_star
        assert np.linalg.norm(beta[k] - b) <= radius(beta[k]) + radius(b)
        assert np.all(beta[k][sup[k] == 0] == 0.0)


@pytest.mark.parametrize("T", [1, 2, 3, 5, 8, 13])
def test_refine_incumbent_trajectory_matches_closed_form(torch_cuda, T):
    """The GPU refinement stopped after T iterations on the separable quadratic
    whose iterates have a closed form (the same case pins the oracle)."""
    from test_oracle_pins import _fista_closed_form, _separable_case
    X, y, l0, l2, M = _separable_case()
    from paper_2602_04551_amd.binding import Context
    ctx = Context(0)
    ctx.set_data(X, y, l0, l2, M, precision="fp64")
    sup = np.array([[1, 1, 0]], np.uint8)
    _, beta, it = ctx.refine_incumbent(sup, np.zeros((1, 3)), tol=0.0, max_iter=T)
    want, _ = _fista_closed_form(T, lambda t: t / (t + 3.0))
    b = beta.cpu().numpy()[0]
    assert it[0].item() == T
    assert np.max(np.abs(b[:2] - want)) <= 1e-13
    assert b[2] == 0.0


def test_bnb_dfs_fp64_trace_identical_to_oracle(torch_cuda, orc):
    inst = datagen.make_instance(35, 11, rho=0.5, k=3, snr=2.0, seed=1, lambda0=0.02, lambda2=0.01)
    o = orc.Oracle.from_instance(inst)
    kw = dict(tol_node=1e-7, max_iter=5000, max_iter_root=20000)
    ref = o.bnb(**kw, trace_cap=100000)
    ctx = ctx_for(inst, "fp64")
    got = ctx.bnb_solve(K=1, policy="dfs", **kw, trace_cap=100000)
    assert got["status"] == 0 and ref["status"] == 0
    assert len(got["trace"]) == len(ref["trace"])
    for a, b in zip(got["trace"], ref["trace"]):
        for f in ("id", "parent", "depth", "branch_j", "decision", "iters", "support_size"):
            assert a[f] == b[f], (f, a, b)
        assert abs(a["lb"] - b["lb"]) <= 1e-10 * max(1.0, abs(b["lb"])) or (a["lb"] == b["lb"])
    assert abs(got["certified"] - ref["certified"]) <= 1e-10 * ref["certified"]
    assert list(got["support"]) == list(ref["support"])


@pytest.mark.parametrize("precision,K", [("fp64", 64), ("fp32", 64), ("fp32", 256), ("bf16", 128), ("fp8", 128)])
def test_bnb_best_first_certifies_the_oracle_optimum(torch_cuda, orc, precision, K):
    inst = datagen.config_instance("C1", seed=0)
    o = orc.Oracle.from_instance(inst)
    ref = o.bnb(tol_node=1e-6, max_iter=2000, max_iter_root=10000)
    ctx = ctx_for(inst, precision)
    got = ctx.bnb_solve(K=K, policy="best", tol_node=1e-6, max_iter=2000, max_iter_root=10000)
    assert got["status"] == 0
    assert abs(got["certified"] - ref["certified"]) <= 1e-8 * ref["certified"]
    assert list(got["support"]) == list(ref["support"])
    assert got["ub"] * (1 - 2e-6) <= got["lb"] <= got["ub"]


def test_edge_cases(torch_cuda, cases):
    from paper_2602_04551_amd.binding import L0L2Error
    inst, o, root = cases["ragged"]
    ctx = ctx_for(inst, "fp64")
    # empty batch
    res = ctx.solve_node_batch(np.zeros((0, inst.p), np.uint8))
    assert res["lb"].numel() == 0
    # everything fixed to zero: the relaxation is 1/2 ||y||^2
    codes = np.full((1, inst.p), FIX0, np.uint8)
    res = ctx.solve_node_batch(codes, tol_node=1e-12, max_iter=20000)
    assert res["lb"].item() == pytest.approx(0.5 * float(inst.y @ inst.y), rel=1e-9)
    # one coordinate
    inst1 = datagen.make_instance(20, 1, k=1, seed=2, M=5.0)
    c1 = ctx_for(inst1, "fp64")
    r1 = c1.solve_node_batch(np.zeros((3, 1), np.uint8), tol_node=1e-9, max_iter=5000)
    assert np.all(r1["status"].cpu().numpy() == 0)
    # invalid arguments surface as errors, not crashes
    with pytest.raises(L0L2Error):
        ctx.solve_node_batch(np.zeros((2, inst.p), np.uint8), max_iter=0)
    with pytest.raises(L0L2Error):
        ctx.set_data(inst.X, inst.y, inst.lambda0, -1.0, inst.M)
    # FP8 storage runs anchored solves only: fixed sweeps are refused
    c8 = ctx_for(inst, "fp8")
    with pytest.raises(L0L2Error):
        c8.admm_sweeps(np.zeros((2, inst.p), np.uint8), np.zeros((2, inst.p), np.float32),
                       np.zeros((2, inst.p), np.float32), 3)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16", "fp8"])
def test_graph_replay_and_eager_issue_agree_bitwise(torch_cuda, cases, precision):
    """Blocks of sweeps replayed from captured HIP graphs and the same blocks
    issued launch by launch (the profiler forces that) give identical bits; a
    rerun of the same batch does too."""
    inst, o, root = cases["wide"]
    K = 70
    codes, beta0, v0 = random_nodes(inst.p, K, 13, root["beta"], root["v"])
    ctx = ctx_for(inst, precision)
    outs = []
    for prof in (False, True, False):
        ctx.profile_enable(prof)
        r = ctx.solve_node_batch(codes, beta0, v0, tol_node=1e-6, max_iter=3000, check_every=10)
        outs.append({k: v.cpu().numpy() for k, v in r.items()})
    ctx.profile_enable(False)
    for other in outs[1:]:
        for k in ("lb", "primal", "iters", "status", "beta", "v"):
            assert np.array_equal(outs[0][k], other[k]), k
