"""The branch-and-bound host logic of the library (csrc/bnb_core.hpp) on the CPU,
with the FP64 oracle plugged in as the node solver: DFS with K = 1 reproduces
the oracle's own depth-first trace exactly, and best-first batches certify the
enumerated optimum."""
import json
import os
import subprocess

import numpy as np
import pytest

from paper_2602_04551_amd import datagen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "bnb_core_check.cpp")


@pytest.fixture(scope="module")
def harness(orc, tmp_path_factory):
    out = str(tmp_path_factory.mktemp("host") / "bnb_core_check")
    odir = os.path.join(ROOT, "oracle")
    subprocess.check_call(["g++", "-O2", "-std=c++17", SRC, "-o", out, f"-L{odir}", "-loracle",
                           f"-Wl,-rpath,{odir}"])
    return out


def run(harness, inst, tmp_path, K, policy, tol=1e-7, root_iter=20000):
    fn = str(tmp_path / "inst.bin")
    with open(fn, "wb") as f:
        np.array([inst.n, inst.p], np.int64).tofile(f)
        np.array([inst.lambda0, inst.lambda2, inst.M], np.float64).tofile(f)
        np.asfortranarray(inst.X).T.ravel().tofile(f)      # column-major
        inst.y.astype(np.float64).tofile(f)
    r = subprocess.run([harness, fn, str(K), str(policy), repr(tol), str(root_iter)], capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr
    lines = [json.loads(s) for s in r.stdout.splitlines()]
    return lines[:-1], lines[-1]


@pytest.mark.parametrize("seed", [0, 1, 3])
def test_dfs_k1_trace_matches_oracle(orc, harness, tmp_path, seed):
    inst = datagen.make_instance(35, 11, rho=0.5, k=3, snr=2.0, seed=seed, lambda0=0.02, lambda2=0.01)
    trace, res = run(harness, inst, tmp_path, K=1, policy=1)
    ref = orc.Oracle.from_instance(inst).bnb(tol_node=1e-7, max_iter=5000, max_iter_root=20000, trace_cap=10**6)
    assert len(trace) == len(ref["trace"])
    for a, b in zip(trace, ref["trace"]):
        for f in ("id", "parent", "depth", "branch_j", "decision", "iters", "support_size"):
            assert a[f] == b[f], (f, a, b)
        assert a["lb"] == b["lb"]
    assert res["certified"] == ref["certified"]
    assert res["solved"] == ref["nodes_solved"] and res["pruned"] == ref["nodes_pruned"]
    assert res["slots_in_use"] == 0


@pytest.mark.parametrize("K", [4, 32])
def test_best_first_batches_certify_the_optimum(orc, harness, tmp_path, K):
    inst = datagen.make_instance(35, 11, rho=0.5, k=3, snr=2.0, seed=2, lambda0=0.02, lambda2=0.01)
    trace, res = run(harness, inst, tmp_path, K=K, policy=0)
    ref = orc.Oracle.from_instance(inst).bnb(tol_node=1e-7, max_iter=5000, max_iter_root=20000)
    assert res["certified"] == pytest.approx(ref["certified"], rel=1e-12)
    assert res["support"] == list(ref["support"])
    assert res["slots_in_use"] == 0
    # every solved node after the root either prunes, closes a leaf or branches
    assert {t["decision"] for t in trace} <= {0, 1, 2, 3}
    ids = [t["id"] for t in trace]
    assert len(ids) == len(set(ids))
