"""Continuous batching with slot refill (l0l2_solve_node_queue): N queued nodes
through K < N slots, a retired node's slot taking the next queued node at the
next block boundary.  Each node's result lands at its own queue position and
equals what the node gets alone: FP64 sweep counts equal to the oracle's and
bounds within 1e-10; reduced modes (anchored from the first sweep) bounds
within 1e-5 of the oracle's.  Per-node sweep budgets retire nodes at their own
count; the batch stays fuller than a fixed batch of the same nodes."""
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


@pytest.fixture(scope="module")
def c1(orc):
    inst = datagen.config_instance("C1", seed=0)
    o = orc.Oracle.from_instance(inst)
    root = o.node_admm(None, tol=1e-7, max_iter=20000)
    return inst, o, root


def nodes(p, N, seed, root, spread=True):
    """N nodes with 1..6 fixings; the warm starts are the root's, perturbed (so
    that sweep counts differ from node to node)."""
    rng = np.random.default_rng(seed)
    codes = np.zeros((N, p), np.uint8)
    for k in range(N):
        idx = rng.choice(p, size=int(rng.integers(1, 7)), replace=False)
        codes[k, idx] = rng.choice([FIX0, FIX1], size=len(idx))
    scale = rng.uniform(0.0, 0.05, size=(N, 1)) if spread else 1e-3
    beta = np.tile(root["beta"], (N, 1)) + scale * rng.normal(size=(N, p))
    v = np.tile(root["v"], (N, 1)) + scale * rng.normal(size=(N, p))
    return codes, beta, v


def ctx_for(inst, precision):
    from paper_2602_04551_amd.binding import Context
    c = Context(0)
    c.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision=precision)
    return c


def test_fp64_queue_matches_the_oracle_node_by_node(torch_cuda, c1):
    inst, o, root = c1
    N, K = 300, 32
    codes, b0, v0 = nodes(inst.p, N, 1, root)
    ctx = ctx_for(inst, "fp64")
    r = ctx.solve_node_queue(codes, b0, v0, K=K, tol_node=1e-7, max_iter=3000, check_every=10)
    lb, pr, it, st = (r[k].cpu().numpy() for k in ("lb", "primal", "iters", "status"))
    gb = r["beta"].cpu().numpy()
    for k in range(0, N, 7):
        ref = o.node_admm(codes[k], b0[k], v0[k], tol=1e-7, max_iter=3000, check_every=10)
        assert it[k] == ref["iters"] and st[k] == ref["status"], k
        assert abs(lb[k] - ref["lb"]) <= 1e-10 * abs(ref["primal"]), k
        assert abs(pr[k] - ref["primal"]) <= 1e-10 * abs(ref["primal"]), k
        assert np.max(np.abs(gb[k] - ref["beta"])) <= 1e-9 * max(1.0, np.max(np.abs(ref["beta"]))), k
    blocks, sparse, node_blocks = ctx.batch_stats()
    # the same nodes in fixed batches of K (each run until its slowest node is
    # done): same sweep counts, but the queue keeps the slots fuller
    fb = fs = fn = 0
    for a in range(0, N, K):
        rb = ctx.solve_node_batch(codes[a:a + K], b0[a:a + K], v0[a:a + K], tol_node=1e-7, max_iter=3000,
                                  check_every=10)
        assert np.array_equal(rb["iters"].cpu().numpy(), it[a:a + K])
        b, sp, nb = ctx.batch_stats()
        fb, fs, fn = fb + b, fs + sp, fn + nb
    occ_queue, occ_fixed = node_blocks / (blocks * K), fn / (fb * K)
    print(f"queue: {blocks} blocks, {sparse} with < 1/8 live, occupancy {occ_queue:.3f}; "
          f"fixed batches: {fb} blocks, {fs} with < 1/8 live, occupancy {occ_fixed:.3f}")
    assert blocks < fb and occ_queue > occ_fixed and sparse <= fs
    ctx.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8"])
def test_reduced_queue_bounds_within_1e5(torch_cuda, c1, precision):
    inst, o, root = c1
    N, K = 160, 32
    codes, b0, v0 = nodes(inst.p, N, 2, root)
    ctx = ctx_for(inst, precision)
    r = ctx.solve_node_queue(codes, b0, v0, K=K, tol_node=1e-6, max_iter=4000, check_every=10)
    lb, pr, st = (r[k].cpu().numpy() for k in ("lb", "primal", "status"))
    assert (st == 0).all()
    assert np.all(lb <= pr)
    for k in range(0, N, 9):
        ref = o.node_admm(codes[k], b0[k], v0[k], tol=1e-6, max_iter=4000, check_every=10)
        assert abs(lb[k] - ref["lb"]) <= 1e-5 * abs(ref["primal"]), k
        assert lb[k] <= ref["primal"] + 1e-12
    ctx.close()


@pytest.mark.parametrize("max_iter", [30, 25])
def test_each_node_retires_at_its_own_budget(torch_cuda, c1, max_iter):
    """A zero tolerance never converges: every node retires at its own budget,
    at the first block boundary at or past it, and the queue still drains."""
    inst, o, root = c1
    N, K = 100, 32
    codes, b0, v0 = nodes(inst.p, N, 3, root)
    ctx = ctx_for(inst, "fp64")
    r = ctx.solve_node_queue(codes, b0, v0, K=K, tol_node=0.0, max_iter=max_iter, check_every=10)
    it, st = r["iters"].cpu().numpy(), r["status"].cpu().numpy()
    assert (st == 1).all()
    assert (it == 10 * ((max_iter + 9) // 10)).all()
    ctx.close()


def test_queue_edge_cases(torch_cuda, c1):
    """N = 0 is a no-op; K >= N runs one batch; K = 1 runs the nodes one by one."""
    inst, o, root = c1
    ctx = ctx_for(inst, "fp64")
    codes, b0, v0 = nodes(inst.p, 5, 4, root)
    r_big = ctx.solve_node_queue(codes, b0, v0, K=64, tol_node=1e-7, max_iter=3000)
    r_one = ctx.solve_node_queue(codes, b0, v0, K=1, tol_node=1e-7, max_iter=3000)
    for k in ("iters", "status"):
        assert np.array_equal(r_big[k].cpu().numpy(), r_one[k].cpu().numpy())
    assert np.max(np.abs(r_big["lb"].cpu().numpy() - r_one["lb"].cpu().numpy())) <= 1e-12
    r0 = ctx.solve_node_queue(np.zeros((0, inst.p), np.uint8), K=8)
    assert r0["lb"].numel() == 0
    ctx.close()
