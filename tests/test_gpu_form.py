"""The b-update form chosen by measurement (Sec. 3.1.1: the p x p D, here as the
Gram form, or the folded Woodbury operand): on the first solve of an instance
where the Gram form is a candidate, one sweep of each form is timed and the
faster kept; the node bounds match the oracle whichever is kept."""
import numpy as np
import pytest

from paper_2602_04551_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("n,p", [(300, 400), (400, 300)])
def test_measured_form_is_the_faster_and_bounds_match(torch_cuda, orc, precision, n, p):
    from paper_2602_04551_amd.binding import Context
    inst = datagen.make_instance(n, p, rho=0.4, k=5, seed=9, lambda0=0.01, lambda2=0.01)
    o = orc.Oracle.from_instance(inst)
    root = o.node_admm(None, tol=1e-7, max_iter=20000)
    rng = np.random.default_rng(3)
    K = 64
    codes = np.zeros((K, p), np.uint8)
    for k in range(K):
        idx = rng.choice(p, size=4, replace=False)
        codes[k, idx] = rng.choice([1, 2], size=4)
    ctx = Context(0)
    ctx.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision=precision)
    assert ctx.bupdate_form()[1:] == (0.0, 0.0)        # not measured before the first solve
    b0 = np.tile(root["beta"], (K, 1))
    v0 = np.tile(root["v"], (K, 1))
    r = ctx.solve_node_batch(codes, b0, v0, tol_node=1e-6, max_iter=4000)
    form, ms_f, ms_g = ctx.bupdate_form()
    assert ms_f > 0 and ms_g > 0
    assert form == ("gram" if ms_g < ms_f else "folded")
    lb, st = r["lb"].cpu().numpy(), r["status"].cpu().numpy()
    for k in range(0, K, 8):
        ref = o.node_admm(codes[k], b0[k], v0[k], tol=1e-6, max_iter=4000)
        assert st[k] == 0
        assert abs(lb[k] - ref["lb"]) <= 1e-5 * abs(ref["primal"])
    print(f"{precision} n={n} p={p}: {form} (folded {ms_f:.4f} ms, gram {ms_g:.4f} ms per sweep)")
    ctx.close()


def test_forms_not_measured_where_they_are_not_candidates(torch_cuda):
    from paper_2602_04551_amd.binding import Context
    inst = datagen.make_instance(100, 300, rho=0.4, k=5, seed=9, lambda0=0.01, lambda2=0.01)   # p > 2 n
    for precision, forced in (("fp32", None), ("fp64", None), ("fp8", None), ("fp32", "gram")):
        ctx = Context(0)
        ctx.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision=precision)
        if forced:
            ctx.set_bupdate_form(forced)
        ctx.solve_node_batch(np.zeros((32, inst.p), np.uint8), tol_node=1e-6, max_iter=3000)
        form, ms_f, ms_g = ctx.bupdate_form()
        assert (ms_f, ms_g) == (0.0, 0.0)
        assert form == (forced or "folded")
        ctx.close()
