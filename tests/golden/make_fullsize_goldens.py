"""Writes the full-size expected values the GPU tests compare against.

Calls only the CPU oracle (oracle/) and the input generator (datagen); nothing
here touches the HIP library.  Three parts, each a separate JSON file under
tests/golden/ so that they can be regenerated independently:

* fullsize_c2_bnb.json -- the n = p = 1000 instance (Toeplitz 0.5, k = 10, SNR 5,
  lambda0 = 0.005, lambda2 = 0.01): the oracle's depth-first branch and bound
  (Alg. 1 with K = 1) to certification, node tolerance 1e-6, eps_prune 2e-6:
  the certified objective, the optimal support and the tree size.
* fullsize_c3_nodes.json -- n = p = 5000 (Toeplitz 0.3, k = 20, SNR 3): the root
  relaxation solved from zero to a 1e-9 gap (20000 sweeps at most), then eight
  nodes of the 4096-node batch (free sets U{50..p}, |F1| U{0..20}, drawn by
  datagen.node_batch_codes with seed 4096) solved from that root to a 1e-6 gap
  (2000 sweeps at most): bound, primal value, sweep count, status.
* fullsize_c5_nodes.json -- n = 1000, p = 50000 (constant correlation 0.2,
  k = 25, SNR 3, lambda0 = 0.002, lambda2 = 0.005): the same with eight nodes of
  the 1024-node batch (seed 1024).

* fullsize_c3_root.npz / fullsize_c5_root.npz -- the oracle's root iterates
  (beta, v) of the two node parts, the warm start the sampled nodes were solved
  from (written with the node part, or alone by the c3root / c5root modes).

Usage: python tests/golden/make_fullsize_goldens.py {c2|c3|c5|c3root|c5root} [workers]
The node parts build one oracle instance, solve the root, then solve the
sampled nodes in `workers` forked processes; c3 and c5 take tens of minutes of
CPU time.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2602_04551_amd import datagen  # noqa: E402

# node slots sampled from each batch: fixed, spread over the batch
SAMPLE = {"C3": (4096, [0, 517, 1023, 1800, 2222, 2900, 3600, 4095]),
          "C5": (1024, [0, 130, 257, 400, 611, 777, 901, 1023])}
ROOT_TOL, ROOT_ITERS = 1e-9, 20000
NODE_TOL, NODE_ITERS, CHECK = 1e-6, 2000, 10


def c2():
    inst = datagen.config_instance("C2", seed=0)
    o = oracle.Oracle.from_instance(inst)
    t0 = time.perf_counter()
    r = o.bnb(tol_node=NODE_TOL, max_iter=NODE_ITERS, max_iter_root=10000, check_every=CHECK, trace_cap=0)
    out = {"workload": "n=1000 p=1000 Toeplitz rho=0.5 k=10 SNR=5 lambda0=0.005 lambda2=0.01 seed 0",
           "oracle": "depth-first branch and bound, K = 1, tol_node 1e-6, eps_prune 2e-6, root 10000 sweeps, "
                     "nodes 2000 sweeps, gap checked every 10",
           "certified": r["certified"], "ub": r["ub"], "status": r["status"],
           "support": [int(j) for j in r["support"]], "nodes_solved": int(r["nodes_solved"]),
           "nodes_pruned": int(r["nodes_pruned"]), "cpu_seconds": round(time.perf_counter() - t0, 1)}
    with open(os.path.join(HERE, "fullsize_c2_bnb.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


_O = None   # the oracle instance, built once and inherited by the forked workers


def _node(args):
    k, codes, beta, v = args
    t0 = time.perf_counter()
    r = _O.node_admm(codes, beta, v, tol=NODE_TOL, max_iter=NODE_ITERS, check_every=CHECK)
    return {"slot": int(k), "lb": r["lb"], "primal": r["primal"], "iters": int(r["iters"]),
            "status": int(r["status"]), "n_free": int(np.sum(codes == 0)), "n_fix1": int(np.sum(codes == 2)),
            "cpu_seconds": round(time.perf_counter() - t0, 1)}


def save_root(name, root):
    np.savez_compressed(os.path.join(HERE, f"fullsize_{name.lower()}_root.npz"), beta=root["beta"], v=root["v"],
                        iters=np.int64(root["iters"]), lb=np.float64(root["lb"]), primal=np.float64(root["primal"]))


def nodes(name, workers, root_only=False):
    global _O
    import multiprocessing as mp
    inst = datagen.config_instance(name, seed=0)
    K, slots = SAMPLE[name]
    t0 = time.perf_counter()
    o = _O = oracle.Oracle.from_instance(inst)
    t_create = time.perf_counter() - t0
    root = o.node_admm(None, tol=ROOT_TOL, max_iter=ROOT_ITERS, check_every=CHECK)
    t_root = time.perf_counter() - t0 - t_create
    print(json.dumps({"root_iters": root["iters"], "root_status": root["status"], "create_s": round(t_create, 1),
                      "root_s": round(t_root, 1)}), flush=True)
    save_root(name, root)
    if root_only:
        return
    codes = datagen.node_batch_codes(inst.p, K, seed=K)
    jobs = [(k, codes[k], root["beta"], root["v"]) for k in slots]
    # fork: the workers share the precomputed instance (this process never uses a GPU)
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_node, jobs)
    out = {"workload": {"C3": "n=p=5000 Toeplitz rho=0.3 k=20 SNR=3 lambda0=0.005 lambda2=0.01 seed 0",
                        "C5": "n=1000 p=50000 constant correlation 0.2 k=25 SNR=3 lambda0=0.002 lambda2=0.005 "
                              "seed 0"}[name],
           "batch": f"datagen.node_batch_codes(p, {K}, seed={K})", "K": K,
           "root": {"lb": root["lb"], "primal": root["primal"], "iters": int(root["iters"]),
                    "status": int(root["status"]), "tol": ROOT_TOL, "max_iter": ROOT_ITERS},
           "node_opts": {"tol": NODE_TOL, "max_iter": NODE_ITERS, "check_every": CHECK},
           "nodes": res, "oracle_create_s": round(t_create, 1), "oracle_root_s": round(t_root, 1)}
    with open(os.path.join(HERE, f"fullsize_{name.lower()}_nodes.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    which = sys.argv[1]
    w = int(sys.argv[2]) if len(sys.argv) > 2 else 4
    if which == "c2":
        c2()
    elif which.endswith("root"):
        nodes(which[:2].upper(), w, root_only=True)
    else:
        nodes(which.upper(), w)
