"""Boundary behaviour of the C ABI on the device: cancellation of a long call
from another thread and before a call, the context staying usable afterwards,
and the library's device-memory accounting returning to where it started when
a context is destroyed."""
import threading
import time

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


def _ctx(inst, precision):
    from paper_2602_04551_amd.binding import Context
    c = Context(0)
    c.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision=precision)
    return c


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_cancel_a_running_node_solve_from_another_thread(torch_cuda, precision):
    """A node solve with a zero tolerance never converges; l0l2_cancel from a
    second thread stops it at a block boundary with L0L2_E_CANCELLED, long
    before its sweep budget, and the next solve on the context runs normally."""
    from paper_2602_04551_amd.binding import L0L2_E_CANCELLED, L0L2Error
    inst = datagen.config_instance("C1", seed=0)
    ctx = _ctx(inst, precision)
    codes = np.zeros((64, inst.p), np.uint8)
    out = {}

    def run():
        t0 = time.perf_counter()
        try:
            ctx.solve_node_batch(codes, tol_node=0.0, max_iter=200000, check_every=10)
            out["rc"] = 0
        except L0L2Error as e:
            out["rc"] = e.code
        out["s"] = time.perf_counter() - t0

    t = threading.Thread(target=run)
    t.start()
    time.sleep(0.3)
    ctx.cancel()
    t.join(timeout=120)
    assert not t.is_alive()
    assert out["rc"] == L0L2_E_CANCELLED, out
    r = ctx.solve_node_batch(codes, tol_node=1e-6, max_iter=5000, check_every=10)
    assert (r["status"].cpu().numpy() == 0).all()
    ctx.close()


def test_cancel_before_a_call_stops_that_call_only(torch_cuda):
    from paper_2602_04551_amd.binding import L0L2_E_CANCELLED, L0L2Error
    inst = datagen.config_instance("C1", seed=0)
    ctx = _ctx(inst, "fp32")
    ctx.cancel()
    with pytest.raises(L0L2Error) as e:
        ctx.bnb_solve(K=16, policy="best", tol_node=1e-6, max_iter=3000, max_iter_root=10000)
    assert e.value.code == L0L2_E_CANCELLED
    r = ctx.bnb_solve(K=16, policy="best", tol_node=1e-6, max_iter=3000, max_iter_root=10000)
    assert r["status"] == 0
    ctx.close()


def test_memory_accounting_returns_to_its_start(torch_cuda):
    """The process-wide count of library-held device bytes is back where it was
    after a context that solved a tree is destroyed; the context's own count
    covers everything it held, and its peak at least that."""
    import gc
    from paper_2602_04551_amd.binding import memory_stats
    gc.collect()   # contexts of earlier tests release their buffers now, not mid-test
    g0, _ = memory_stats()
    inst = datagen.config_instance("C1", seed=0)
    ctx = _ctx(inst, "bf16")
    ctx.bnb_solve(K=32, policy="best", tol_node=1e-6, max_iter=3000, max_iter_root=10000)
    held, peak = ctx.memory_stats()
    g1, _ = memory_stats()
    assert 0 < held <= peak
    assert g1 - g0 == held
    ctx.close()
    g2, _ = memory_stats()
    assert g2 == g0
