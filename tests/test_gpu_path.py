"""The lambda0 path (Sec. 4.1, selection of lambda0): branch and bound over a
decreasing lambda0 grid on one instance, each point warm-started from the
previous one (its certified support seeds the incumbent, its root iterates
start the root), with the precompute done once.

* l0l2_lambda0_max equals minus the smallest forward score of App. A.2 at the
  empty support with lambda0 = 0, evaluated by the oracle; just below it the
  optimum is no longer empty and at it the empty support is certified.
* At every grid point the certified objective and support equal the oracle's
  depth-first branch and bound run from scratch at that lambda0, and equal a
  cold GPU solve at that point (the warm start changes the tree, not the
  optimum).
"""
import numpy as np
import pytest

from paper_2602_04551_amd import datagen

pytestmark = pytest.mark.gpu
KW = dict(K=32, policy="best", tol_node=1e-6, max_iter=3000, max_iter_root=10000)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ctx(inst, precision):
    from paper_2602_04551_amd.binding import Context
    c = Context(0)
    c.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision=precision)
    return c


def test_lambda0_max_is_the_first_forward_gain(torch_cuda, orc):
    inst = datagen.config_instance("C1", seed=0)
    ctx = _ctx(inst, "fp64")
    lmax = ctx.lambda0_max()
    o0 = orc.Oracle(inst.X, inst.y, 0.0, inst.lambda2, inst.M)
    delta, _ = o0.mp_deltas(np.zeros(inst.p, np.uint8), np.zeros(inst.p), inst.y)
    assert abs(lmax - (-delta.min())) <= 1e-13 * lmax
    # at lambda0_max the empty support is optimal; a little below it, it is not
    ctx.set_penalties(lmax * 1.001)
    r = ctx.bnb_solve(**KW)
    assert r["status"] == 0 and len(r["support"]) == 0
    ctx.set_penalties(lmax * 0.95)
    r = ctx.bnb_solve(**KW)
    assert r["status"] == 0 and len(r["support"]) >= 1
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_path_matches_the_oracle_and_cold_solves(torch_cuda, orc, precision):
    inst = datagen.config_instance("C1", seed=0)
    ctx = _ctx(inst, precision)
    lmax = ctx.lambda0_max()
    grid = lmax * 0.6 ** np.arange(1, 6)
    path = ctx.bnb_path(grid, **KW)
    assert len(path) == len(grid)
    nodes_warm = sum(r["nodes_solved"] for r in path)
    nodes_cold = 0
    for lam, r in zip(grid, path):
        o = orc.Oracle(inst.X, inst.y, float(lam), inst.lambda2, inst.M)
        ref = o.bnb(tol_node=1e-6, max_iter=3000, max_iter_root=10000)
        assert r["status"] == 0
        assert abs(r["certified"] - ref["certified"]) <= 1e-8 * abs(ref["certified"]), lam
        assert list(r["support"]) == list(ref["support"]), lam
        ctx.set_penalties(float(lam))
        cold = ctx.bnb_solve(**KW)
        nodes_cold += cold["nodes_solved"]
        assert list(cold["support"]) == list(r["support"])
        assert abs(cold["certified"] - r["certified"]) <= 1e-12 * abs(r["certified"])
    print(f"{precision}: supports {[len(r['support']) for r in path]}, nodes warm {nodes_warm} cold {nodes_cold}")
    ctx.close()


def test_penalties_are_validated_and_the_precompute_is_kept(torch_cuda):
    from paper_2602_04551_amd.binding import L0L2Error
    inst = datagen.config_instance("C1", seed=0)
    ctx = _ctx(inst, "fp64")
    r0 = ctx.bnb_solve(**KW)
    for bad in ((-1.0, 0.01, 1.0), (0.01, 0.0, 1.0), (0.01, 0.01, -2.0), (float("nan"), 0.01, 1.0)):
        with pytest.raises(L0L2Error):
            ctx.set_penalties(*bad)
    ctx.set_penalties(inst.lambda0, inst.lambda2, inst.M)
    r1 = ctx.bnb_solve(**KW)
    assert r1["certified"] == r0["certified"] and list(r1["support"]) == list(r0["support"])
    ctx.close()
