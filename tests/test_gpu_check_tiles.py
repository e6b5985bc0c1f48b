"""The FP64 bound (Prop. 1 with the rounding margin) on both tile shapes of the
exact check: a batch large enough for the 64 x 64 tiles (n = p = 2048, 1024
nodes: 16 node tiles of 64 against 64 row tiles) and a 64-node slice of it,
which takes the 32 x 32 tiles.  Every node's bound agrees between the two
launches to 1e-12 relative (the tiles only change the summation order of the
two products), and sampled nodes agree with the oracle's bound to the same bar.
A whole FP64 batch of that size, whose gap checks run on the 64 x 64 tiles,
stops its sampled nodes after the oracle's number of sweeps.
"""
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


def test_bound_on_wide_and_narrow_check_tiles_matches_the_oracle(torch_cuda, orc):
    from paper_2602_04551_amd.binding import Context
    n = p = 2048
    K = 1024
    inst = datagen.make_instance(n, p, rho=0.3, k=12, seed=21, lambda0=0.01, lambda2=0.05)
    rng = np.random.default_rng(8)
    codes = np.zeros((K, p), np.uint8)
    for k in range(K):
        idx = rng.choice(p, size=int(rng.integers(0, 40)), replace=False)
        codes[k, idx] = rng.choice([FIX0, FIX1], size=len(idx))
    b = rng.normal(scale=0.05, size=(K, p))
    ctx = Context(0)
    ctx.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision="fp64")
    lb_wide = ctx.dual_bound(codes, b).cpu().numpy()
    lb_narrow = ctx.dual_bound(codes[:64], b[:64]).cpu().numpy()
    ctx.close()
    assert np.all(np.isfinite(lb_wide))
    scale = np.maximum(1.0, np.abs(lb_wide[:64]))
    assert np.max(np.abs(lb_wide[:64] - lb_narrow) / scale) <= 1e-12
    o = orc.Oracle.from_instance(inst, factor="numpy")
    for k in list(range(0, K, 97)) + [K - 1]:
        r = inst.y - inst.X @ b[k]
        ref = o.dual_bound(codes[k], r)
        print(f"node {k}: gpu {lb_wide[k]:.15e} oracle {ref:.15e}")
        assert abs(lb_wide[k] - ref) <= 1e-12 * max(1.0, abs(ref)), k


def test_fp64_batch_on_wide_check_tiles_takes_the_oracles_decisions(torch_cuda, orc):
    """A 1024-node FP64 batch at n = p = 2048 runs its gap checks on the 64 x 64
    tiles; sampled nodes stop after the oracle's number of sweeps, with its
    status, and their bounds agree with the oracle's to 1e-10 of the primal."""
    from paper_2602_04551_amd.binding import Context
    n = p = 2048
    K = 1024
    inst = datagen.make_instance(n, p, rho=0.3, k=12, seed=22, lambda0=0.01, lambda2=0.05)
    rng = np.random.default_rng(9)
    codes = np.zeros((K, p), np.uint8)
    for k in range(K):
        idx = rng.choice(p, size=int(rng.integers(1, 30)), replace=False)
        codes[k, idx] = rng.choice([FIX0, FIX1], size=len(idx))
    ctx = Context(0)
    ctx.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision="fp64")
    r = ctx.solve_node_batch(codes, None, None, tol_node=1e-6, max_iter=600, check_every=10)
    it, st, lb = r["iters"].cpu().numpy(), r["status"].cpu().numpy(), r["lb"].cpu().numpy()
    ctx.close()
    o = orc.Oracle.from_instance(inst, factor="numpy")
    for k in (0, 511, K - 1):
        ref = o.node_admm(codes[k], None, None, tol=1e-6, max_iter=600, check_every=10)
        print(f"node {k}: gpu {it[k]} sweeps, status {st[k]}, lb {lb[k]:.15e}; "
              f"oracle {ref['iters']}, {ref['status']}, {ref['lb']:.15e}")
        assert it[k] == ref["iters"] and st[k] == ref["status"], k
        assert abs(lb[k] - ref["lb"]) <= 1e-10 * abs(ref["primal"]), k
