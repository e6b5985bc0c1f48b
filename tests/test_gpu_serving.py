"""Serving: whole branch-and-bound solves of several instances of different
sizes admitted under an HBM budget and run concurrently, their blocks of ADMM
sweeps batched across instances into shared launches by the server's executor.
Each result is the same alone and in the mix, bit for bit, and the same with
batching across instances on and off (server contexts take their tile shapes
from a size rule, and a grouped tile computes what the instance's own launch
would), admitted instances overlap in time, the budget caps the concurrent
footprint, each request's device high-water mark stays within its admission
estimate, and queued or running requests can be cancelled."""
import json
import os
import time

import numpy as np
import pytest

from paper_2602_04551_amd import datagen

pytestmark = pytest.mark.gpu

KW = dict(K=32, policy="best", tol_node=1e-6, max_iter=3000, max_iter_root=10000)
SIZES = [(60, 30, 0), (120, 45, 1), (90, 60, 2), (200, 40, 3), (150, 70, 4), (80, 35, 5)]


@pytest.fixture(scope="module")
def instances():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return [datagen.make_instance(n, p, rho=0.3, k=3, snr=3.0, seed=s, lambda0=0.02, lambda2=0.01)
            for n, p, s in SIZES]


@pytest.fixture(scope="module")
def alone(instances):
    """Each instance through a server that runs one request at a time, with
    batching across instances off (its own captured blocks on its own stream)."""
    from paper_2602_04551_amd.binding import Server
    srv = Server(0, hbm_budget_bytes=0, max_concurrent=1, batching=False, **KW)
    out = []
    for inst in instances:
        rid = srv.submit(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision="fp32")
        out.append(srv.wait(rid, timeout_s=600))
    srv.close()
    return out


def overlaps(res):
    iv = sorted((r["admit_s"], r["done_s"]) for r in res)
    return any(iv[i + 1][0] < iv[i][1] for i in range(len(iv) - 1))


def test_results_identical_alone_and_in_the_mix(instances, alone, orc):
    from paper_2602_04551_amd.binding import Server
    srv = Server(0, hbm_budget_bytes=0, max_concurrent=3, **KW)
    ids = []
    for i, inst in enumerate(instances):
        ids.append(srv.submit(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision="fp32"))
        if i == 2:
            time.sleep(0.05)     # later arrivals join while the first ones run
    res = [srv.wait(r, timeout_s=600) for r in ids]
    srv.close()
    for a, b in zip(res, alone):
        assert a["status"] == 0
        for key in ("certified", "ub", "lb", "nodes_solved", "nodes_pruned", "batches"):
            assert a[key] == b[key], key
        assert list(a["support"]) == list(b["support"])
        assert np.array_equal(a["beta"], b["beta"])
        assert 0 < a["peak_bytes"] <= a["footprint_bytes"]
    assert overlaps(res)
    ref = orc.Oracle.from_instance(instances[1]).bnb(tol_node=1e-6, max_iter=3000, max_iter_root=10000)
    assert abs(res[1]["certified"] - ref["certified"]) <= 1e-8 * ref["certified"]
    assert list(res[1]["support"]) == list(ref["support"])


def _same(a, b):
    assert a["status"] == b["status"] == 0
    for key in ("certified", "ub", "lb", "nodes_solved", "nodes_pruned", "batches"):
        assert a[key] == b[key], key
    assert list(a["support"]) == list(b["support"])
    assert np.array_equal(a["beta"], b["beta"])


def _serve(insts, precs, batching, max_concurrent, **kw):
    from paper_2602_04551_amd.binding import Server
    srv = Server(0, hbm_budget_bytes=0, max_concurrent=max_concurrent, batching=batching, **kw)
    ids = [srv.submit(i.X, i.y, i.lambda0, i.lambda2, i.M, precision=pr) for i, pr in zip(insts, precs)]
    res = [srv.wait(r, timeout_s=600) for r in ids]
    st = srv.batching_stats()
    srv.close()
    return res, st


@pytest.mark.parametrize("precisions", [("fp32", "fp64"), ("bf16",)])
def test_batching_across_instances_at_n_p_1000(instances, precisions):
    """Three n = p = 1000 instances (the benchmark's configuration with three
    seeds) in FP32 and FP64 mode (six requests at once), and in BF16 mode
    (three requests, the split-form register-tile kernels): their blocks share
    launches (more than one instance per grouped launch on average) and every
    result equals, bit for bit, the instance solved alone with batching off
    (its own captured blocks on its own stream); the seed-0 instance's certified
    value and support equal the oracle's (tests/golden/fullsize_c2_bnb.json)."""
    big = [datagen.config_instance("C2", seed=s) for s in (0, 1, 2)]
    insts = [i for i in big for _ in precisions]
    precs = [pr for _ in big for pr in precisions]
    alone_res, _ = _serve(insts, precs, False, 1, **KW)
    mix_res, st = _serve(insts, precs, True, len(insts), **KW)
    print(f"batching stats {st}: {st['members'] / max(st['launches'], 1):.2f} instances per shared launch")
    assert st["launches"] > 0 and st["members"] > st["launches"]
    for a, b in zip(mix_res, alone_res):
        _same(a, b)
    with open(os.path.join(os.path.dirname(__file__), "golden", "fullsize_c2_bnb.json")) as f:
        ref = json.load(f)
    for r in mix_res[:len(precisions)]:
        assert abs(r["certified"] - ref["certified"]) <= 1e-8 * ref["certified"]
        assert list(r["support"]) == ref["support"]


def test_batching_more_instances_than_a_group_holds(instances, alone):
    """Twelve requests at once (two copies of each small instance): groups hold
    at most eight members, so rounds split into several launches per kind;
    every result equals the alone run."""
    insts = instances + instances
    res, st = _serve(insts, ["fp32"] * len(insts), True, len(insts), **KW)
    assert st["launches"] > 0
    for a, b in zip(res, alone + alone):
        _same(a, b)


def test_budget_caps_concurrent_footprint(instances, alone):
    from paper_2602_04551_amd.binding import Server, lib
    fp = [lib.l0l2_footprint_bytes(i.n, i.p, 1, KW["K"]) for i in instances]
    budget = int(max(fp) * 1.5)
    srv = Server(0, hbm_budget_bytes=budget, max_concurrent=4, **KW)
    ids = [srv.submit(i.X, i.y, i.lambda0, i.lambda2, i.M, precision="fp32") for i in instances]
    res = [srv.wait(r, timeout_s=600) for r in ids]
    srv.close()
    for a, b in zip(res, alone):
        assert a["certified"] == b["certified"]
    # at every admission instant the running footprints fit in the budget
    for r in res:
        t = r["admit_s"]
        running = sum(x["footprint_bytes"] for x in res if x["admit_s"] <= t < x["done_s"])
        assert running <= budget
    # arrival order is kept
    admits = [r["admit_s"] for r in res]
    assert admits == sorted(admits)


def test_oversized_request_is_rejected(instances):
    from paper_2602_04551_amd.binding import L0L2Error, Server
    srv = Server(0, hbm_budget_bytes=1 << 20, max_concurrent=1, **KW)
    inst = instances[0]
    with pytest.raises(L0L2Error):
        srv.submit(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M)
    srv.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16", "fp8"])
def test_footprint_estimate_covers_a_solve(instances, precision):
    """The admission estimate bounds what a whole solve holds on the device: the
    free device memory drops by at most l0l2_footprint_bytes between before the
    context exists and the end of a BnB solve on n = p = 1000 with K = 256
    (instance copies, batch workspace, the Gram form's G where it applies,
    captured graphs, the warm-start pool)."""
    import torch
    from paper_2602_04551_amd.binding import Context, lib
    inst = datagen.config_instance("C2", seed=0)
    code = {"fp64": 0, "fp32": 1, "bf16": 2, "fp8": 3}[precision]
    est = lib.l0l2_footprint_bytes(inst.n, inst.p, code, 256)
    torch.zeros(1, device="cuda")   # the runtime's own first-use memory is not the solve's
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0 = torch.cuda.mem_get_info()[0]
    c = Context(0)
    c.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision=precision)
    r = c.bnb_solve(K=256, policy="best", tol_node=1e-6, max_iter=2000, max_iter_root=10000)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    used = free0 - torch.cuda.mem_get_info()[0]
    held, peak = c.memory_stats()
    c.close()
    assert r["status"] == 0
    print(f"{precision}: held after {used / 2**20:.1f} MiB, library peak {peak / 2**20:.1f} MiB, "
          f"estimate {est / 2**20:.1f} MiB")
    # the high-water mark of the library's own buffers (transients of set_data and
    # of the solve included), and what stays on the device, within the estimate
    assert held <= peak <= est
    assert used <= est


def test_cancel_queued_and_running_requests(instances):
    """A queued request cancelled ends at once with L0L2_E_CANCELLED; a running
    one ends cancelled or (if it finished first) certified; the others are
    unaffected."""
    from paper_2602_04551_amd.binding import L0L2_E_CANCELLED, L0L2Error, Server
    big = datagen.config_instance("C2", seed=0)
    srv = Server(0, hbm_budget_bytes=0, max_concurrent=1, **KW)
    r0 = srv.submit(big.X, big.y, big.lambda0, big.lambda2, big.M, precision="fp64")
    r1 = srv.submit(instances[0].X, instances[0].y, instances[0].lambda0, instances[0].lambda2, instances[0].M)
    r2 = srv.submit(instances[1].X, instances[1].y, instances[1].lambda0, instances[1].lambda2, instances[1].M)
    srv.cancel(r1)
    time.sleep(0.05)
    srv.cancel(r0)
    with pytest.raises(L0L2Error) as e:
        srv.wait(r1, timeout_s=60)
    assert e.value.code == L0L2_E_CANCELLED
    try:
        a = srv.wait(r0, timeout_s=600)
        assert a["status"] == 0
    except L0L2Error as e0:
        assert e0.code == L0L2_E_CANCELLED
    b = srv.wait(r2, timeout_s=600)
    assert b["status"] == 0
    with pytest.raises(L0L2Error):
        srv.cancel(r2)    # already collected
    srv.close()


def test_destroy_releases_a_waiting_thread(instances):
    """Destroying the server while another thread waits (without a time limit)
    on a queued request: the waiter returns L0L2_E_CANCELLED, nothing hangs."""
    import threading
    from paper_2602_04551_amd.binding import L0L2_E_CANCELLED, L0L2Error, Server
    big = datagen.config_instance("C2", seed=0)
    srv = Server(0, hbm_budget_bytes=0, max_concurrent=1, **KW)
    srv.submit(big.X, big.y, big.lambda0, big.lambda2, big.M, precision="fp64")
    rq = srv.submit(instances[2].X, instances[2].y, instances[2].lambda0, instances[2].lambda2, instances[2].M)
    got = {}

    def waiter():
        try:
            got["res"] = srv.wait(rq)
        except L0L2Error as e:
            got["code"] = e.code

    t = threading.Thread(target=waiter)
    t.start()
    time.sleep(0.1)
    srv.close()
    t.join(timeout=120)
    assert not t.is_alive()
    assert got.get("code") == L0L2_E_CANCELLED or got.get("res", {}).get("status") == 0
