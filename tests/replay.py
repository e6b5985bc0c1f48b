"""Replay of a branch-and-bound trace by the CPU oracle (test infrastructure).

Given the trace of a GPU solve (nodes in the order the host processed them,
with their decisions), the oracle re-solves every node of that tree itself:
the same fixings (F0, F1), warm-started from the oracle's own solution of the
parent (the root from zero), and takes each decision of Alg. 1 against the
same incumbent value UB the GPU run had at that point.  Only the tree shape
and the UB sequence come from the trace; every number the decisions are
compared with is the oracle's.

Decisions are compared where the oracle's margins clear a tolerance band:
* prune: |LB_eff - UB (1 - eps)| >= prune_band * UB;
* rounding: every free coordinate has |z_j - 1/2| >= z_band;
* branching: the gap between the best and the second-best floored score
  min(z, 1 - z) is >= score_band (when every free score is 0: the gap between
  the two largest |beta_j| relative to the largest is >= score_band).
Decisions inside a band are counted and returned, never silently accepted.
For an in-band branching decision the GPU's index must still be a free
coordinate, and the oracle-side score deficit of that index (the oracle's best
floored score minus its score at the GPU's index; with every free score 0, the
relative |beta| deficit) is returned as its maximum over the tree.
"""
from __future__ import annotations

import math

import numpy as np

FREE, FIX0, FIX1 = 0, 1, 2
GRID = 1048576.0   # 2^20: the branching score grid


def node_codes(trace, p):
    """Fixing codes and path keys of every node of the trace.  Node ids are
    allocated in pairs when a node is branched: the z = 0 child first (odd id),
    then the z = 1 child (even id).  The path key lists (j, code) from the root
    down; it identifies the node and its chain of warm starts."""
    branch_of = {r["id"]: r["branch_j"] for r in trace if r["decision"] == 0}
    codes = {0: np.zeros(p, np.uint8)}
    keys = {0: ()}
    parent = {r["id"]: r["parent"] for r in trace}

    def get(i):
        if i in codes:
            return codes[i]
        par = parent[i]
        c = get(par).copy()
        j, f = branch_of[par], (FIX0 if i % 2 == 1 else FIX1)
        c[j] = f
        codes[i] = c
        keys[i] = keys[par] + ((int(j), f),)
        return c

    for r in trace:
        get(r["id"])
    return codes, keys, parent


def _scores(o, codes, beta):
    """Free coordinates' z and floored branching scores (the oracle's z)."""
    import oracle
    free = np.flatnonzero(codes == FREE)
    z = np.array([oracle.z(beta[j], FREE, o.lambda0, o.lambda2, o.M) for j in free]) if len(free) else np.zeros(0)
    sc = np.floor(np.minimum(z, 1.0 - z) * GRID)
    return free, z, sc


def replay(o, trace, *, tol_node, max_iter, max_iter_root, check_every, eps_prune, prune_band=1e-5,
           z_band=1e-6, score_band=2.0 ** -20, fista_tol=1e-12, fista_max_iter=1000, cache=None):
    """Returns a dict of counts: compared / mismatched / in-band per decision kind,
    plus lists describing each mismatch."""
    p = o.p
    codes, keys, parent = node_codes(trace, p)
    state = {}        # node id -> (beta, v, lb_eff) of the oracle's own solve
    cache = {} if cache is None else cache
    out = {k: 0 for k in ("prune_cmp", "prune_band", "branch_cmp", "branch_band", "support_cmp", "support_band",
                          "ub_cmp", "solved", "select_cmp", "select_band")}
    out["mismatch"] = []
    out["band_deficit_max"] = 0.0
    ub_before = math.inf
    for rec in trace:
        i, d = rec["id"], rec["decision"]
        c = codes[i]
        if d == 3:
            # pruned at selection on the bound inherited from the parent
            lbi = state[parent[i]][2]
            thr = ub_before * (1.0 - eps_prune)
            if abs(lbi - thr) >= prune_band * abs(ub_before):
                out["select_cmp"] += 1
                if not lbi >= thr:
                    out["mismatch"].append(("select", i, lbi, thr))
            else:
                out["select_band"] += 1
            ub_before = rec["ub_global"]
            continue
        key = keys[i]
        if key in cache:
            r, mask, ub_o, j_o = cache[key]
        else:
            if i == 0:
                beta0, v0, mi = None, None, max_iter_root
            else:
                beta0, v0, mi = state[parent[i]][0], state[parent[i]][1], max_iter
            r = o.node_admm(c, beta0, v0, tol=tol_node, max_iter=mi, check_every=check_every)
            mask, _ = o.support(c, r["beta"])
            ub_o, _, _ = o.fista(mask, r["beta"], tol=fista_tol, max_iter=fista_max_iter)
            j_o = o.branch(c, r["beta"])
            cache[key] = (r, mask, ub_o, j_o)
        out["solved"] += 1
        lb_inh = -math.inf if i == 0 else state[parent[i]][2]
        lb_eff = max(r["lb"], lb_inh)
        state[i] = (r["beta"], r["v"], lb_eff)
        thr = ub_before * (1.0 - eps_prune)
        pruned_o = math.isfinite(ub_before) and lb_eff >= thr
        if not math.isfinite(ub_before) or abs(lb_eff - thr) >= prune_band * abs(ub_before):
            out["prune_cmp"] += 1
            if pruned_o != (d == 1):
                out["mismatch"].append(("prune", i, lb_eff, thr, d))
                ub_before = rec["ub_global"]
                continue
        else:
            out["prune_band"] += 1
        if d == 1 or pruned_o:
            ub_before = rec["ub_global"]
            continue
        # rounding: the support (and with it the incumbent value) where no z sits near 1/2
        free, z, sc = _scores(o, c, r["beta"])
        if len(free) == 0 or np.min(np.abs(z - 0.5)) >= z_band:
            out["support_cmp"] += 1
            if rec["support_size"] != int(mask.sum()):
                out["mismatch"].append(("support", i, rec["support_size"], int(mask.sum())))
            else:
                out["ub_cmp"] += 1
                if abs(rec["ub_node"] - ub_o) > 1e-8 * abs(ub_o):
                    out["mismatch"].append(("ub", i, rec["ub_node"], ub_o))
        else:
            out["support_band"] += 1
        # branching
        gpu_j = rec["branch_j"] if d == 0 else -1
        if len(free) == 0:
            out["branch_cmp"] += 1
            if gpu_j != -1 or j_o != -1:
                out["mismatch"].append(("leaf", i, gpu_j, j_o))
        else:
            if sc.max() > 0:
                top = np.sort(sc)[::-1]
                margin = (top[0] - (top[1] if len(top) > 1 else -1.0)) / GRID
            else:
                ab = np.sort(np.abs(r["beta"][free]))[::-1]
                margin = (ab[0] - (ab[1] if len(ab) > 1 else 0.0)) / max(ab[0], 1e-300)
            if margin >= score_band:
                out["branch_cmp"] += 1
                if gpu_j != j_o:
                    out["mismatch"].append(("branch", i, gpu_j, j_o, margin))
            else:
                out["branch_band"] += 1
                if d == 0:
                    pos = np.flatnonzero(free == gpu_j)
                    if len(pos) == 0:
                        out["mismatch"].append(("branch_not_free", i, gpu_j))
                    elif sc.max() > 0:
                        deficit = (sc.max() - sc[pos[0]]) / GRID
                        out["band_deficit_max"] = max(out["band_deficit_max"], float(deficit))
                    else:
                        ab = np.abs(r["beta"][free])
                        deficit = (ab.max() - ab[pos[0]]) / max(ab.max(), 1e-300)
                        out["band_deficit_max"] = max(out["band_deficit_max"], float(deficit))
        ub_before = rec["ub_global"]
    return out
