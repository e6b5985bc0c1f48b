"""The allocation-free refinement entry point (l0l2_refine_incumbent_noalloc)
against the allocating one (l0l2_refine_incumbent), through the C ABI.

Both run the same refinement kernel on the same inputs, so their outputs must
be bit-identical; the allocation-free one keeps its residual rows in the
library's fixed device scratch, which every call on the device shares.  Two
calls in a row, the second with a smaller batch (and other supports), check
that nothing of the first call's scratch contents leaks into the second.
Supports wider than 64 coordinates take the kernel's streamed path, the one
that uses the scratch; narrower ones (and the empty support) are mixed in.
"""
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


def _supports(rng, K, p, lo, hi):
    sup = np.zeros((K, p), np.uint8)
    for k in range(K):
        size = 0 if k == 0 else int(rng.integers(lo, hi + 1))
        sup[k, rng.choice(p, size=size, replace=False)] = 1
    return sup


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_refinement_equals_the_allocating_entry_point(torch_cuda, precision):
    torch = torch_cuda
    from paper_2602_04551_amd.binding import Context
    inst = datagen.make_instance(700, 300, rho=0.5, k=20, snr=5.0, seed=3)
    ctx = Context(0)
    ctx.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision=precision)
    dev, p = ctx.torch_device, inst.p
    rng = np.random.default_rng(11)
    for K, lo, hi in ((40, 20, 200), (7, 1, 120)):
        print(f"[noalloc] {precision} K={K} support sizes {lo}..{hi}", flush=True)
        sup = _supports(rng, K, p, lo, hi)
        start = (0.3 * rng.standard_normal((K, p))).astype(np.float64 if precision == "fp64" else np.float32)
        sup_d = torch.from_numpy(sup).to(dev)
        start_d = torch.from_numpy(start).to(dev)
        # outputs allocated by the caller beforehand, poisoned so that a missing write shows
        beta_out = torch.full((K, p), float("nan"), dtype=torch.float64, device=dev)
        obj = torch.full((K,), float("nan"), dtype=torch.float64, device=dev)
        iters = torch.full((K,), -7, dtype=torch.int32, device=dev)
        ctx.refine_incumbent_noalloc(sup_d, start_d, beta_out, obj, iters, tol=1e-12, max_iter=1000)
        torch.cuda.synchronize()
        obj_ref, beta_ref, it_ref = ctx.refine_incumbent(sup_d, start_d, tol=1e-12, max_iter=1000)
        torch.cuda.synchronize()
        assert torch.equal(obj, obj_ref), (obj - obj_ref).abs().max().item()
        assert torch.equal(beta_out, beta_ref)
        assert torch.equal(iters, it_ref)
        assert bool(torch.isfinite(obj).all())
        assert int(sup.sum(axis=1).max()) > 64      # the streamed path (the scratch) was exercised


def test_noalloc_refinement_rejects_a_batch_beyond_its_scratch(torch_cuda):
    torch = torch_cuda
    from paper_2602_04551_amd.binding import Context, L0L2Error, L0L2_E_INVALID
    inst = datagen.make_instance(700, 40, rho=0.5, k=5, snr=5.0, seed=4)
    ctx = Context(0)
    ctx.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision="fp64")
    K = (32 << 20) // (8 * 768) + 1          # one row more than 32 MiB of residual rows at padded n = 768
    dev = ctx.torch_device
    sup = torch.zeros((K, inst.p), dtype=torch.uint8, device=dev)
    start = torch.zeros((K, inst.p), dtype=torch.float64, device=dev)
    beta_out = torch.zeros((K, inst.p), dtype=torch.float64, device=dev)
    obj = torch.zeros(K, dtype=torch.float64, device=dev)
    with pytest.raises(L0L2Error) as e:
        ctx.refine_incumbent_noalloc(sup, start, beta_out, obj)
    assert e.value.code == L0L2_E_INVALID
    # one row fewer fits and runs (every support empty: objective 1/2 ||y||^2)
    ctx.refine_incumbent_noalloc(sup[:K - 1], start[:K - 1], beta_out[:K - 1], obj[:K - 1])
    torch.cuda.synchronize()
    assert torch.allclose(obj[:K - 1], torch.full_like(obj[:K - 1], 0.5 * float(inst.y @ inst.y)), rtol=1e-14)
