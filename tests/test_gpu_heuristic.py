"""Matching-pursuit root heuristic (Sec. 3.5; App. A.2 scores) on the GPU
against the oracle.

Every GPU move is replayed on the oracle's side: at the state before the move
(the GPU's support and coefficients, the residual y - X beta recomputed by the
oracle), the oracle scores every coordinate; the GPU's move must be of the
step's kind and carry the oracle's smallest score, unless another coordinate
lies within the band of it (then the choice is counted as in band and must
still be a move with a negative score).  A step the GPU left empty must have no
oracle score below -band.  Where no decision is in band, the move sequence,
support and coefficients equal the oracle's own run.  Band (a reading): the
scores are differences of F of size |F| computed from n-term FP64 sums in
another order, so they agree to about n u |F|; 1e-12 |F| covers n <= 1000.
"""
import json
import os

import numpy as np
import pytest

from paper_2602_04551_amd import datagen

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ctx(inst, precision="fp64"):
    from paper_2602_04551_amd.binding import Context
    c = Context(0)
    c.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision=precision)
    return c


def _replay(o, X, y, moves, max_moves, band):
    """Walk the rounds of forward / backward steps with the GPU's moves and check
    each step against the oracle's scores at that state; returns (in-band
    choices, final mask, final beta)."""
    p = X.shape[1]
    mask = np.zeros(p, np.uint8)
    beta = np.zeros(p)
    t = in_band = 0
    while t < max_moves:
        moved = False
        for want in (0, 1):          # 0: forward (j outside S), 1: backward (j in S)
            if t >= max_moves:
                break
            delta, bnew = o.mp_deltas(mask, beta, y - X @ beta)
            cand = np.flatnonzero(((mask != 0) == want) & (delta < 0.0))
            best = delta[cand].min() if cand.size else np.inf
            took = t < len(moves) and ((moves[t] < 0) == bool(want))
            if not took:
                # the GPU found no move in this step: nor may the oracle, beyond the band
                assert best >= -band, (t, want, best)
                continue
            j = abs(moves[t]) - 1
            assert ((mask[j] != 0) == bool(want)) and delta[j] < 0.0, (t, j, delta[j])
            if delta[j] != best:
                assert delta[j] - best <= band, (t, j, delta[j], best)
                in_band += 1
            beta[j] = 0.0 if want else bnew[j]
            mask[j] = 0 if want else 1
            t += 1
            moved = True
        if not moved:
            break
    assert t == len(moves)
    return in_band, mask, beta


@pytest.mark.parametrize("cfg", ["C1", "C2"])
def test_matching_pursuit_moves_replay_on_the_oracle(torch_cuda, orc, cfg):
    inst = datagen.config_instance(cfg, seed=0)
    o = orc.Oracle.from_instance(inst)
    ctx = _ctx(inst)
    mask_g, beta_g, obj_g, moves_g = ctx.matching_pursuit()
    ctx.close()
    mask_o, beta_o, moves_o = o.matching_pursuit(max_moves=4 * min(inst.n, inst.p))
    F_o = o.objective(mask_o, beta_o)
    band = 1e-12 * abs(F_o)
    assert len(moves_g) > 0
    in_band, mask_r, beta_r = _replay(o, inst.X, inst.y, moves_g, 4 * min(inst.n, inst.p), band)
    np.testing.assert_array_equal(mask_r, mask_g)
    np.testing.assert_allclose(beta_g, beta_r, rtol=0, atol=1e-10 * max(1.0, np.abs(beta_r).max()))
    assert abs(obj_g - o.objective(mask_g, beta_g)) <= 1e-12 * abs(F_o)
    print(f"{cfg}: {len(moves_g)} moves, {in_band} in band, F = {obj_g:.12g}")
    if in_band == 0:
        assert moves_g == moves_o
        np.testing.assert_array_equal(mask_g, mask_o)
        np.testing.assert_allclose(beta_g, beta_o, rtol=0, atol=1e-10 * max(1.0, np.abs(beta_o).max()))
        assert abs(obj_g - F_o) <= 1e-12 * abs(F_o)


def test_matching_pursuit_move_budget_and_no_move_case(torch_cuda, orc):
    """max_moves cuts the run after exactly that many moves (the oracle's first
    moves); lambda0 above every first-step gain leaves the support empty."""
    inst = datagen.config_instance("C1", seed=0)
    o = orc.Oracle.from_instance(inst)
    ctx = _ctx(inst)
    _, _, _, full = ctx.matching_pursuit()
    assert len(full) > 3
    mask, beta, obj, moves = ctx.matching_pursuit(max_moves=3)
    assert moves == full[:3]
    assert int(mask.sum()) == sum(1 if m > 0 else -1 for m in moves)
    ctx.close()
    big = datagen.config_instance("C1", seed=0)
    big.lambda0 = 10.0
    ctx = _ctx(big)
    mask, beta, obj, moves = ctx.matching_pursuit()
    assert moves == [] and mask.sum() == 0 and not beta.any()
    assert abs(obj - 0.5 * float(big.y @ big.y)) <= 1e-14
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_bnb_with_the_root_heuristic_certifies_the_same_optimum(torch_cuda, orc, precision):
    """Seeding the incumbent with the heuristic's support changes the tree, not
    the certified optimum (n = p = 1000: the committed oracle result)."""
    inst = datagen.config_instance("C2", seed=0)
    with open(os.path.join(GOLD, "fullsize_c2_bnb.json")) as f:
        gold = json.load(f)
    ctx = _ctx(inst, precision)
    kw = dict(K=256, policy="best", tol_node=1e-6, max_iter=2000, max_iter_root=10000)
    r0 = ctx.bnb_solve(**kw)
    r1 = ctx.bnb_solve(root_heuristic=True, **kw)
    ctx.close()
    for r in (r0, r1):
        assert r["status"] == 0
        assert list(r["support"]) == gold["support"]
        assert abs(r["certified"] - gold["certified"]) <= 1e-8 * abs(gold["certified"])
    print(f"{precision}: nodes {r0['nodes_solved']} -> {r1['nodes_solved']}, "
          f"{r0['seconds']:.3f} s -> {r1['seconds']:.3f} s")
