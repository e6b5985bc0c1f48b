"""Benchmark of the batched node-relaxation hot path on one MI355X.

Headline workload (the batching configuration, the largest that the benchmark
runs on one GPU at full size): n = p = 5000, Toeplitz rho = 0.3, k = 20 unit
spikes, SNR = 3, lambda0 = 0.005, lambda2 = 0.01, node batches of 4096 whose
nodes keep f ~ U{50..p} free coordinates (|F1| ~ U{0..20}, the rest fixed to
zero), warm-started from the root relaxation.  The mixed path multiplies with
X in BF16 (FP32 accumulation, FP32 state, FP64 bounds and incumbent
objective); the FP32 and FP64 GPU paths run the same batches.  One step = one
pass of the whole hot path over one batch: warm-start assembly, ADMM to the
node tolerance with the FP64 gap checks and rigorous bounds, rounding and
branching, FP64 incumbent refinement, and the host's prune / branch decisions.
Inputs are synthetic and resident on the GPU before timing starts.

Also in the same JSON line: time-to-certified-optimum of the full branch and
bound on the n = p = 1000 instance in every precision, node batches of the
n = 1000, p = 50000 (FP8 storage) workload, and the CPU oracle timed on a
32-node sample of the headline batch.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# dense MFMA TFLOP/s, MI355X; FP8 storage widens its codes to BF16, so its products run at the BF16 rate
PEAK = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0, "fp8": 2500.0}
METRIC = "node relaxations/s + time-to-certified-optimum, mixed vs FP64 GPU path"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--K", type=int, default=4096, help="nodes per batch of the headline workload")
    ap.add_argument("--no-ttco", action="store_true", help="skip the n = p = 1000 branch-and-bound runs")
    ap.add_argument("--heuristic-study", action="store_true",
                    help="branch and bound with and without the matching-pursuit root incumbent")
    ap.add_argument("--heur-seconds", type=float, default=20.0,
                    help="time limit of the n = 1000, p = 50 000 runs of --heuristic-study")
    ap.add_argument("--no-highdim", action="store_true", help="skip the n = 1000, p = 50000 node batches")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-sample", type=int, default=128, help="nodes of the headline batch the oracle solves")
    ap.add_argument("--only-mixed", action="store_true", help="headline precision only (short profiled runs)")
    ap.add_argument("--batching", action="store_true",
                    help="n = p = 5000 node batches of 512..4096 (free sets U[50, p]), BF16 vs FP32")
    ap.add_argument("--serve", action="store_true",
                    help="Poisson stream of independent instances through the server: p50/p99 TTCO")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-concurrent", type=int, default=8, help="instances in flight at once")
    ap.add_argument("--serve-config", choices=["c4", "reduced"], default="c4")
    ap.add_argument("--serve-precision", default="fp32")
    ap.add_argument("--serve-K", type=int, default=64, help="node batch of each instance's branch and bound")
    ap.add_argument("--serve-limit", type=float, default=60.0, help="per-request time limit (censored beyond)")
    ap.add_argument("--serve-solo", type=int, default=4, help="draws timed alone to set the arrival rate")
    ap.add_argument("--serve-interarrival", type=float, default=0.0, help="mean inter-arrival time (0: measured)")
    ap.add_argument("--serve-batching", choices=["on", "off", "both"], default="on")
    ap.add_argument("--serve-oracle", action="store_true",
                    help="CPU oracle time to certify the smallest draws of the serving stream (no GPU)")
    ap.add_argument("--serve-oracle-count", type=int, default=8)
    ap.add_argument("--serve-oracle-nodes", type=int, default=2000, help="node cap of each oracle run")
    ap.add_argument("--highdim", action="store_true",
                    help="n = 1000, p = 50000 node batches of 256 and 1024: FP8, BF16, FP32 vs FP64")
    ap.add_argument("--node-parallel", action="store_true",
                    help="the node-parallel study: n = 3000, p in {1e4, 3e4, 1e5}, K in {1, 10, 50, 100}, "
                         "branch and bound under a time limit: nodes/s, gap and peak device memory vs K")
    ap.add_argument("--np-seconds", type=float, default=10.0, help="time limit of each node-parallel run")
    ap.add_argument("--np-p", type=str, default="10000,30000,100000")
    ap.add_argument("--np-precision", type=str, default="fp64")
    ap.add_argument("--np-tol", type=float, default=1e-4, help="node gap tolerance of the study (the paper's 1e-4)")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/hbm_traffic.json from two rocprofv3 counter CSVs (FETCH_SIZE, WRITE_SIZE) "
                         "of a --copy-calibrate run of the headline, then exit")
    ap.add_argument("--traffic-workload", default="c3")
    ap.add_argument("--bf16-rows", type=int, default=128, choices=[128, 256],
                    help="rows of the single-term BF16 sweep's largest tile")
    ap.add_argument("--traffic-families", default="",
                    help="comma-separated sweep families to summarise (default: every family found)")
    ap.add_argument("--copy-calibrate", action="store_true",
                    help="first dispatch one device copy of 256 MiB, the reference for HBM counter scaling")
    return ap.parse_args()


HEADLINE = ("C3", "n=p=5000 Toeplitz rho=0.3 k=20 SNR=3 lambda0=0.005 lambda2=0.01, node batches of {K} "
                  "(free sets U{{50..p}}, |F1| U{{0..20}}, warm-started from the root), X products in BF16 "
                  "with FP32 accumulation and FP32 state, FP64 bounds and incumbent objective")


def fp64_root(inst, tol=1e-9, max_iter=20000):
    """Root relaxation solved once in FP64 on the GPU (the warm start every precision
    shares), its rounded incumbent refined in FP64: (beta, v, UB, sweeps)."""
    from paper_2602_04551_amd.binding import Context
    ctx = Context(0)
    ctx.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision="fp64")
    p = inst.p
    z = np.zeros((1, p), np.uint8)
    r = ctx.solve_node_batch(z, tol_node=tol, max_iter=max_iter)
    obj, _, _ = ctx.refine_incumbent(ctx.round_branch(z, r["beta"])["support"], r["beta"])
    out = (r["beta"][0].cpu().numpy(), r["v"][0].cpu().numpy(), float(obj[0].item()), int(r["iters"][0].item()))
    ctx.close()
    return out


class Path:
    """One precision of the hot path on one instance's node batch (same codes and
    the same FP64 root warm start for every precision)."""

    def __init__(self, inst, precision, codes, root):
        import torch
        from paper_2602_04551_amd.binding import Context
        self.torch = torch
        self.inst, self.precision = inst, precision
        self.K = codes.shape[0]
        self.ctx = Context(0)
        t0 = time.perf_counter()
        self.ctx.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, rho=1.0, precision=precision)
        torch.cuda.synchronize()
        self.set_data_s = time.perf_counter() - t0
        rb, rv, self.ub, _ = root
        dev, dt = self.ctx.torch_device, self.ctx.state_dtype
        self.codes = torch.from_numpy(np.ascontiguousarray(codes)).to(dev)
        self.beta0 = torch.from_numpy(rb).to(dev, dt).expand(self.K, inst.p).contiguous()
        self.v0 = torch.from_numpy(rv).to(dev, dt).expand(self.K, inst.p).contiguous()
        torch.cuda.synchronize()
        self.step()   # settles the tile shapes and captured graphs outside any timed region
        torch.cuda.synchronize()

    def step(self):
        """Whole hot path over the batch; returns (node-iterations, pruned, branched)."""
        c = self.ctx
        res = c.solve_node_batch(self.codes, self.beta0, self.v0, tol_node=1e-6, max_iter=2000, check_every=10)
        rb = c.round_branch(self.codes, res["beta"])
        obj, _, fit = c.refine_incumbent(rb["support"], res["beta"])
        self.detail = (res["iters"], rb["support_size"], fit, res["status"])
        lb = res["lb"].cpu().numpy()
        ub = obj.cpu().numpy()
        bj = rb["branch_j"].cpu().numpy()
        iters = int(res["iters"].sum().item())
        UB = min(self.ub, float(ub.min()))
        thr = UB * (1.0 - 2e-6)
        pruned = int(np.sum(lb >= thr))
        branched = int(np.sum((lb < thr) & (bj >= 0)))
        return iters, pruned, branched

    def close(self):
        self.ctx.close()


# --- CPU baseline: the oracle on a sample of the headline batch --------------

_CPU = None   # (oracle instance, codes, root beta, root v), inherited by the forked workers


def _cpu_nodes(args):
    """One worker: the oracle as it stands on its share of the sample (node solve,
    rounding, branching, refinement), until `seconds` of work have passed."""
    idx, seconds = args
    o, codes, rb, rv = _CPU
    t0 = time.perf_counter()
    done = sweeps = 0
    for k in idx:
        r = o.node_admm(codes[k], rb, rv, tol=1e-6, max_iter=2000, check_every=10)
        mask, _ = o.support(codes[k], r["beta"])
        o.branch(codes[k], r["beta"])
        o.fista(mask, r["beta"])
        done += 1
        sweeps += r["iters"]
        if time.perf_counter() - t0 >= seconds:
            break
    return done, sweeps, time.perf_counter() - t0


def _cpu_baseline_proc(cfg, K, sample, rb, rv, seconds, workers, conn):
    """Runs in a spawned process that never touches the GPU: builds the oracle's
    instance once (its once-per-tree factor from numpy's LAPACK, which the timing
    leaves out), then forks `workers` single-threaded oracle processes that
    share it and solve the sampled nodes."""
    global _CPU
    import multiprocessing as mp
    import oracle
    from paper_2602_04551_amd import datagen
    inst = datagen.config_instance(cfg, seed=0)
    codes = datagen.node_batch_codes(inst.p, K, seed=K)
    t0 = time.perf_counter()
    o = oracle.Oracle.from_instance(inst, factor="numpy")
    t_factor = time.perf_counter() - t0
    slots = np.linspace(0, K - 1, sample).round().astype(int)
    _CPU = (o, codes, rb, rv)
    shares = [list(slots[i::workers]) for i in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_cpu_nodes, [(s, seconds) for s in shares if s])
    conn.send({"res": res, "wall": time.perf_counter() - t0, "factor_s": t_factor})
    conn.close()


def cpu_model():
    """The host CPU as lscpu names it (model name, sockets, cores), else /proc/cpuinfo's model name."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    name = info.get("Model name")
    if not name:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        name = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    parts = [name or "unknown"]
    for k in ("Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)"):
        if k in info:
            parts.append(f"{k} {info[k]}")
    return ", ".join(parts)


def cpu_baseline(cfg, K, root, seconds, sample):
    """The CPU oracle on `sample` nodes spread over the headline batch (same codes,
    same warm start), node-parallel over the host's cores."""
    import multiprocessing as mp
    nproc = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = nproc
    # at most 16 worker processes: the share of host CPUs that comes with one GPU here
    workers = max(1, min(avail, 16, sample))
    ctx = mp.get_context("spawn")
    a, b = ctx.Pipe(duplex=False)
    pr = ctx.Process(target=_cpu_baseline_proc, args=(cfg, K, sample, root[0], root[1], seconds, workers, b))
    pr.start()
    msg = a.recv()
    pr.join()
    res = msg["res"]
    done = sum(d for d, _, _ in res)
    sweeps = sum(s for _, s, _ in res)
    busy = max(t for _, _, t in res)
    per_core = done / sum(t for _, _, t in res)
    return dict(value=round(done / busy, 3), unit="node relaxations/s", cores=len(res), kind="oracle",
                per_core_value=round(per_core, 4), cpu_model=cpu_model(), nproc=nproc, affinity=avail,
                sample=f"{done} of {sample} nodes spread over the {K}-node batch (same codes, same FP64 root "
                       f"warm start), {sweeps} ADMM sweeps in all, each node solved to the 1e-6 gap, rounded, "
                       f"branched and refined by the single-threaded FP64 oracle; {len(res)} worker processes "
                       f"(at most 16: the host CPU share of one GPU) ran for {busy:.1f} s at most; the oracle's "
                       f"once-per-tree factor (X^T X + rho I)^-1 came from numpy in {msg['factor_s']:.1f} s, "
                       f"not timed")


def b_update_info(ctx):
    """The b-update form the library measured and kept for the instance (Sec. 3.1.1)."""
    form, ms_f, ms_g = ctx.bupdate_form()
    return {"form": form, "measured_ms_per_sweep": {"folded": round(ms_f, 4), "gram": round(ms_g, 4)},
            "note": "Gram form b = (w - G w) / rho with G = Xh^T Xh (2 p^2 flops per node-sweep) against the "
                    "folded operand Xh = L^-1 X (two contractions, 4 n p); timed once per instance on the batch"}


def batch_detail(path):
    """Per-node work of the last step: ADMM sweeps, support sizes, refinement iterations."""
    sw, ss, fi, st = (t.cpu().numpy().astype(np.float64) for t in path.detail)
    return {"admm_sweeps_mean": round(float(sw.mean()), 2), "admm_sweeps_max": int(sw.max()),
            "converged": int((st == 0).sum()), "nodes": int(len(st)),
            "support_mean": round(float(ss.mean()), 2), "support_max": int(ss.max()),
            "fista_iters_mean": round(float(fi.mean()), 2), "fista_iters_max": int(fi.max())}


def kernel_source_digest():
    """SHA-256 over the sources that define the kernels and their launches: every
    header, and every HIP file that defines a kernel (host-only files, such as
    the ABI wrappers and the server, do not count)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for fn in sorted(glob.glob(os.path.join(ROOT, "paper_2602_04551_amd", "csrc", "*"))):
        if fn.endswith((".hip", ".hpp")):
            with open(fn, "rb") as f:
                text = f.read()
            if fn.endswith(".hpp") or b"__global__" in text:
                h.update(text)
    return h.hexdigest()


TRAFFIC_FILE = "hbm_traffic.json"


def measured_traffic(kname, workload):
    """HBM bytes per launch of a contraction family on a workload from the
    committed counter summary (rocprofv3 FETCH_SIZE + WRITE_SIZE passes), or None
    when there is none or the kernel sources have changed since it was taken."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(workload)
    if not rec or kernel_source_digest() != rec.get("source_digest"):
        return None
    return rec["per_launch_bytes"].get(kname)


# library kernel families and the kernel names that belong to them
FAMILIES = {"admm_xtu.bf16": ("k_admm_xtu_bf16", "k_admm_xtu_anch_bf16"),
            "admm_xtu.f32": ("k_admm_xtu<float", "k_admm_xtu_lds<float", "k_admm_xtu_anch"),
            "admm_xtu.f64": ("k_admm_xtu<double", "k_admm_xtu_lds<double")}


def traffic_summary(fetch_csv, write_csv, workload, last=50, families=None):
    """HBM bytes per launch of each sweep family from two rocprofv3 counter
    passes of the same command: FETCH_SIZE and WRITE_SIZE (KiB per dispatch),
    scaled by what each reads for the 256 MiB device copy dispatched first
    (--copy-calibrate), averaged over the family's last `last` dispatches (the
    benchmark's last step; the tile tuner's masked launches come earlier)."""
    import csv
    import re

    def load(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        return rows

    out = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = load(path, counter)
        # the calibration copy is the first copy dispatched (later copies, such as
        # the measured copy rate's, move other amounts)
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        ref = copies[0] * 1024.0 if copies else None
        scale = (256.0 * 2 ** 20) / ref if ref else 1.0
        for fam, pats in FAMILIES.items():
            if families and fam not in families:
                continue
            vals = [float(r["Counter_Value"]) * 1024.0 * scale for r in rows
                    if any(re.search(re.escape(pt), r["Kernel_Name"]) for pt in pats)]
            if vals:
                v = vals[-last:]
                out.setdefault(fam, {})[counter] = (sum(v) / len(v), len(v), scale)
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILE)
    allw = json.load(open(path)) if os.path.exists(path) else {}
    allw[workload] = {
        "what": "HBM bytes per launch of each sweep family: FETCH_SIZE + WRITE_SIZE, each scaled so that the "
                "256 MiB device copy dispatched first reads 256 MiB, averaged over the family's last dispatches "
                "(the benchmark's last step); valid for the kernel sources of the digest",
        "source_digest": kernel_source_digest(),
        "per_launch_bytes": {f: round(v["FETCH_SIZE"][0] + v["WRITE_SIZE"][0]) for f, v in out.items()
                             if "FETCH_SIZE" in v and "WRITE_SIZE" in v},
        "fetch_bytes": {f: round(v["FETCH_SIZE"][0]) for f, v in out.items() if "FETCH_SIZE" in v},
        "write_bytes": {f: round(v["WRITE_SIZE"][0]) for f, v in out.items() if "WRITE_SIZE" in v},
        "dispatches": {f: v["FETCH_SIZE"][1] for f, v in out.items() if "FETCH_SIZE" in v},
        "scale": {c: next(iter(out.values()))[c][2] for c in ("FETCH_SIZE", "WRITE_SIZE") if out}}
    with open(path, "w") as f:
        json.dump(allw, f, indent=1)
    print(json.dumps(allw[workload]))


def roofline(prof, n, p, workload=None):
    """Dominant sweep contraction by measured time; achieved = algorithmic flops
    (2 n p per active node-iteration; the Gram form's 2 p^2 equals it at n = p)
    over its summed launch durations.  traffic: the counter figure for that
    kernel on `workload` when one is committed for the current sources."""
    sweep = [k for k in prof if k.startswith(("gemm_xw", "admm_xtu")) and prof[k][0] > 0]
    kname = max(sweep, key=lambda k: prof[k][1])
    launches, ms, units = prof[kname]
    prec = kname.split(".")[1]
    achieved = 2.0 * n * p * units / (ms * 1e-3) / 1e12
    traffic = measured_traffic(kname, workload) if workload else None
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK[prec], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK[prec], 4), "traffic": traffic,
            "traffic_unit": f"HBM bytes per launch (rocprofv3 counters, profiles/{TRAFFIC_FILE})",
            "kernel": kname,
            "launches": launches, "avg_us": round(1e3 * ms / max(launches, 1), 3),
            "flops_per_launch": round(2.0 * n * p * units / max(launches, 1)),
            "node_iterations": units}
    kernels = {k: {"launches": v[0], "ms": round(v[1], 3), "node_iterations": v[2]} for k, v in prof.items()
               if v[0] > 0}
    return roof, kernels


def run_path(path, steps, warmup):
    """Timed steps with the library in its default mode (blocks of sweeps
    replayed from HIP graphs), then a separate pass with per-launch HIP-event
    timing (launches issued one by one) for the kernel durations."""
    torch = path.torch
    for _ in range(warmup):
        path.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = 0
    for _ in range(steps):
        i, _, _ = path.step()
        its += i
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    path.ctx.profile_enable(True)
    for _ in range(max(1, min(steps, 3))):
        path.step()
    torch.cuda.synchronize()
    prof = {k: path.ctx.profile_query(k) for k in path.ctx.KERNELS}
    path.ctx.profile_enable(False)
    return dt, its, prof


# bytes per element of the stored folded operand: FP8 codes, BF16 hi + lo, FP32, FP64
X_BYTES = {"fp8": 1, "bf16": 4, "fp32": 4, "fp64": 8}


def sweep_bytes_roofline(prof, n, p, prec):
    """HBM view of the sweeps: algorithmic bytes of a sweep = the stored operand
    streamed once per contraction (2 n p b_X) plus the node state read and
    written once per active node (beta and V in FP32, 16 p) and its codes
    (p / 4 at two bits), over the summed durations of both contractions."""
    fam = {"fp8": "fp8", "bf16": "bf16", "fp32": "f32", "fp64": "f64"}[prec]
    xw, xtu = prof.get("gemm_xw." + fam, (0, 0.0, 0)), prof.get("admm_xtu." + fam, (0, 0.0, 0))
    sweeps, units = xw[0], xw[2]
    ms = xw[1] + xtu[1]
    if sweeps == 0 or ms <= 0:
        return None
    nbytes = sweeps * 2.0 * n * p * X_BYTES[prec] + units * (16.0 * p + p / 4.0)
    achieved = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
            "frac": round(achieved / 8000.0, 4), "sweeps": sweeps,
            "node_iterations": units, "kernels": ["gemm_xw." + fam, "admm_xtu." + fam]}


def node_batch_run(inst, prec, K, root, profile=True):
    """One node batch of the workload (free sets U{50..p}, |F1| U{0..20}, seed K),
    warm-started from the shared FP64 root: one untimed solve (tiles, graphs),
    one timed, one with per-launch HIP-event timing."""
    import torch
    from paper_2602_04551_amd import datagen
    from paper_2602_04551_amd.binding import Context
    n, p = inst.n, inst.p
    ctx = Context(0)
    t0 = time.perf_counter()
    ctx.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision=prec)
    torch.cuda.synchronize()
    sd = time.perf_counter() - t0
    codes = torch.from_numpy(datagen.node_batch_codes(p, K, seed=K)).to(ctx.torch_device)
    b0 = torch.from_numpy(root[0]).to(ctx.torch_device, ctx.state_dtype).expand(K, p).contiguous()
    v0 = torch.from_numpy(root[1]).to(ctx.torch_device, ctx.state_dtype).expand(K, p).contiguous()
    ctx.solve_node_batch(codes, b0, v0, tol_node=1e-6, max_iter=2000)     # warm-up, tiles, graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.solve_node_batch(codes, b0, v0, tol_node=1e-6, max_iter=2000)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    it = r["iters"].cpu().numpy()
    run = {"value": round(K / dt, 2), "seconds": round(dt, 4), "iters_mean": round(float(it.mean()), 2),
           "iters_max": int(it.max()), "converged": int((r["status"] == 0).sum().item()),
           "set_data_s": round(sd, 3), "b_update": b_update_info(ctx)["form"]}
    blocks, sparse, node_blocks = ctx.batch_stats()
    run["blocks"] = {"total": blocks, "under_1_8_live": sparse,
                     "occupancy": round(node_blocks / max(1, blocks * ((K + 31) // 32 * 32)), 4)}
    if profile:
        ctx.profile_enable(True)
        ctx.solve_node_batch(codes, b0, v0, tol_node=1e-6, max_iter=2000)
        prof = {k: ctx.profile_query(k) for k in ctx.KERNELS}
        ctx.profile_enable(False)
        run["roofline"], run["kernels"] = roofline(prof, n, p)
        run["roofline_hbm"] = sweep_bytes_roofline(prof, n, p, prec)
    ctx.close()
    print(json.dumps({f"{prec}_K{K}": run["value"]}), file=sys.stderr, flush=True)
    return run


def node_queue_run(inst, prec, N, K, root):
    """N nodes of the workload (free sets U{50..p}, |F1| U{0..20}, seed N) through K
    slots refilled as nodes retire (l0l2_solve_node_queue), from the shared FP64
    root: one untimed run (tiles, graphs, form), one timed."""
    import torch
    from paper_2602_04551_amd import datagen
    from paper_2602_04551_amd.binding import Context
    n, p = inst.n, inst.p
    ctx = Context(0)
    ctx.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision=prec)
    codes = torch.from_numpy(datagen.node_batch_codes(p, N, seed=N)).to(ctx.torch_device)
    b0 = torch.from_numpy(root[0]).to(ctx.torch_device, ctx.state_dtype).expand(N, p).contiguous()
    v0 = torch.from_numpy(root[1]).to(ctx.torch_device, ctx.state_dtype).expand(N, p).contiguous()
    ctx.solve_node_queue(codes[:K], b0[:K], v0[:K], K=K, tol_node=1e-6, max_iter=2000)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.solve_node_queue(codes, b0, v0, K=K, tol_node=1e-6, max_iter=2000)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    blocks, sparse, node_blocks = ctx.batch_stats()
    it = r["iters"].cpu().numpy()
    ctx.close()
    out = {"value": round(N / dt, 2), "seconds": round(dt, 4), "queue": N, "slots": K,
           "iters_mean": round(float(it.mean()), 2), "iters_max": int(it.max()),
           "converged": int((r["status"] == 0).sum().item()),
           "blocks": {"total": blocks, "under_1_8_live": sparse,
                      "occupancy": round(node_blocks / max(1, blocks * ((K + 31) // 32 * 32)), 4)}}
    print(json.dumps({f"{prec}_queue{N}_K{K}": out["value"]}), file=sys.stderr, flush=True)
    return out


def node_batch_runs(inst, Ks, precs, workload, label):
    """Node-batch throughput on one instance, one batch per K and precision."""
    out = {"metric": f"node relaxations/s ({label} workload)", "unit": "node relaxations/s",
           "config": {"workload": workload, "node_tol": 1e-6,
                      "warm_start": "root relaxation solved once in FP64 to a 1e-9 gap, shared by all precisions"},
           "runs": {}}
    root = fp64_root(inst)
    for prec in precs:
        for K in Ks:
            out["runs"][f"{prec}_K{K}"] = node_batch_run(inst, prec, K, root)
    print(json.dumps(out), flush=True)


def batching_main(args):
    """n = p = 5000 batches, K in {512, 1024, 2048, 4096}: BF16 split sweeps against FP32; then
    the autotuner's batch axis (node-sweeps per second for K = 32 .. 4096) in both precisions."""
    from paper_2602_04551_amd import datagen
    from paper_2602_04551_amd.binding import Context
    inst = datagen.config_instance("C3", seed=0)
    node_batch_runs(inst, (512, 1024, 2048, 4096), ("bf16", "fp32"),
                    "n=p=5000 Toeplitz rho=0.3 k=20 SNR=3 lambda0=0.005 lambda2=0.01, node batches with free sets "
                    "U{50..p}, |F1| U{0..20}", "batching")
    tuning = {}
    for prec in ("bf16", "fp32"):
        ctx = Context(0)
        ctx.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision=prec)
        k_t, rates = ctx.tune_batch_size(k_max=4096, frac=0.9)
        tuning[prec] = {"chosen_K": k_t, "node_sweeps_per_s": {str(k): round(v) for k, v in rates.items()}}
        ctx.close()
    print(json.dumps({"batch_tuning": tuning}), flush=True)


def highdim_main(args):
    """n = 1000, p = 50000 (constant correlation 0.2), K in {256, 1024}: FP32 and BF16 split
    sweeps against the FP64 path."""
    from paper_2602_04551_amd import datagen
    inst = datagen.config_instance("C5", seed=0)
    node_batch_runs(inst, (256, 1024), ("fp32", "bf16", "fp8", "fp64"),
                    "n=1000 p=50000 constant correlation 0.2 k=25 SNR=3 lambda0=0.002 lambda2=0.005, node batches "
                    "with free sets U{50..p}, |F1| U{0..20}", "high-dimensional")


def mp_lambda0(ctx, k0, ratio=0.8, steps=60):
    """lambda0 for a study instance (a reading of Sec. 4.1's tuning, which runs
    the branch and bound along a path and keeps the lambda0 whose support best
    matches the truth): the largest lambda0 on the grid lambda0_max ratio^i at
    which the matching-pursuit support (Sec. 3.5) holds at least k0 coordinates."""
    lmax = ctx.lambda0_max()
    lam = lmax
    for _ in range(steps):
        lam *= ratio
        ctx.set_penalties(lam)
        mask = ctx.matching_pursuit()[0]
        if int(mask.sum()) >= k0:
            return lam, int(mask.sum()), lmax
    return lam, int(mask.sum()), lmax


def node_parallel_main(args):
    """Sec. 4.4's node-parallel study rerun on synthetic data: branch and bound
    with batches of K in {1, 10, 50, 100} under a time limit on n = 3000
    instances with p in {1e4, 3e4, 1e5}: nodes per second, the gap reached, and
    the peak device memory of the library's buffers relative to K = 1."""
    import torch
    from paper_2602_04551_amd import datagen
    from paper_2602_04551_amd.binding import Context
    out = {"metric": "node-parallel study (nodes/s and peak device memory vs batch size K)",
           "config": {"workload": "n=3000 constant correlation 0.2 k=10 SNR=10/3, lambda2 = lambda2* (ridge on the "
                                  "true support), M = 1.5 x ridge max, lambda0 by the matching-pursuit rule; "
                                  f"best-first branch and bound, {args.np_seconds:g} s per run, "
                                  f"{args.np_precision} path, node tolerance {args.np_tol:g}",
                      "time_limit_s": args.np_seconds, "precision": args.np_precision, "node_tol": args.np_tol},
           "runs": {}}
    for p in [int(v) for v in args.np_p.split(",")]:
        inst = datagen.node_parallel_instance(p)
        ctx = Context(0)
        t0 = time.perf_counter()
        ctx.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision=args.np_precision)
        torch.cuda.synchronize()
        sd = time.perf_counter() - t0
        lam, k_mp, lmax = mp_lambda0(ctx, 10)
        rows = {}
        for K in (1, 10, 50, 100):
            ctx.memory_stats(reset_peak=True)
            r = ctx.bnb_solve(K=K, policy="best", tol_node=args.np_tol, max_iter=2000, max_iter_root=10000,
                              time_limit_s=args.np_seconds)
            held, peak = ctx.memory_stats()
            gap = (r["ub"] - r["lb"]) / abs(r["ub"]) if np.isfinite(r["ub"]) and r["ub"] != 0 else None
            rows[str(K)] = {"nodes": r["nodes_solved"], "seconds": round(r["seconds"], 3),
                            "nodes_per_s": round(r["nodes_solved"] / max(r["seconds"], 1e-9), 2),
                            "gap": gap, "status": r["status"], "peak_gb": round(peak / 1e9, 3),
                            "support_size": len(r["support"])}
            print(json.dumps({"p": p, "K": K, **rows[str(K)]}), file=sys.stderr, flush=True)
        base = rows["1"]
        for K, v in rows.items():
            v["nodes_per_s_vs_K1"] = round(v["nodes_per_s"] / max(base["nodes_per_s"], 1e-9), 2)
            v["peak_vs_K1"] = round(v["peak_gb"] / base["peak_gb"], 3)
        out["runs"][str(p)] = {"n": inst.n, "lambda0": lam, "lambda0_max": lmax, "mp_support": k_mp,
                               "lambda2": inst.lambda2, "M": inst.M, "set_data_s": round(sd, 3), "by_K": rows}
        ctx.close()
    print(json.dumps(out), flush=True)


def heuristic_main(args):
    """Branch and bound with and without the matching-pursuit incumbent (Sec. 3.5,
    App. A.2) seeded before the root: n = p = 1000 to certification, and
    n = 1000, p = 50 000 under a time limit (gap reached, incumbent value,
    nodes), in the mixed BF16 and the FP64 paths."""
    import torch
    from paper_2602_04551_amd import datagen
    from paper_2602_04551_amd.binding import Context
    out = {"metric": "branch and bound with / without the matching-pursuit root incumbent", "runs": {}}
    for cfg, K, limit in (("C2", 256, 0.0), ("C5", 256, args.heur_seconds)):
        inst = datagen.config_instance(cfg, seed=0)
        for prec in ("bf16", "fp64"):
            ctx = Context(0)
            ctx.set_data(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision=prec)
            if cfg == "C2":    # settle tiles and graphs
                ctx.bnb_solve(K=K, policy="best", tol_node=1e-6, max_iter=2000, max_iter_root=10000)
            row = {}
            for heur in (False, True):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = ctx.bnb_solve(K=K, policy="best", tol_node=1e-6, max_iter=2000, max_iter_root=10000,
                                  time_limit_s=limit, root_heuristic=heur)
                torch.cuda.synchronize()
                gap = (r["ub"] - r["lb"]) / abs(r["ub"]) if np.isfinite(r["ub"]) and r["ub"] != 0 else None
                row["heuristic" if heur else "plain"] = {
                    "seconds": round(time.perf_counter() - t0, 3), "status": r["status"], "ub": r["ub"],
                    "lb": r["lb"], "gap": gap, "nodes": r["nodes_solved"], "support_size": len(r["support"])}
                print(json.dumps({"cfg": cfg, "prec": prec, "heuristic": heur,
                                  **row["heuristic" if heur else "plain"]}), file=sys.stderr, flush=True)
            ctx.close()
            out["runs"][f"{cfg}_{prec}"] = {"n": inst.n, "p": inst.p, "K": K, "time_limit_s": limit, **row}
    print(json.dumps(out), flush=True)


def serve_main(args):
    """The serving stream: independent instances arriving as a Poisson process
    through the server (admission under an HBM budget of 80 % of the free device
    memory, node solves of the admitted instances batched into shared launches).
    c4: 64 draws of n ~ U{500..5000}, p ~ U{1000..20000}, Toeplitz rho ~ U[0, 0.7],
    k ~ U{5..30}, SNR ~ U[2, 10], lambda0 = 0.005, lambda2 = 0.01 (datagen.
    serving_instance, seed 0); reduced: n ~ U{500..2000}, p ~ U{1000..4000},
    k ~ U{5..12}.  The mean inter-arrival time is half the mean solo time to
    certified optimum of the first --serve-solo draws (measured first, one at a
    time, batching on) unless --serve-interarrival gives it.  Per request: time
    to certified optimum (submit to done) with a per-request limit; requests that
    hit it are censored (their time counts at the limit) and reported as such.
    --serve-batching both runs the stream with batching across instances on and
    then off."""
    import torch
    from paper_2602_04551_amd import datagen
    from paper_2602_04551_amd.binding import Server
    rng = np.random.default_rng(0)
    reqs = []
    t_gen = time.perf_counter()
    for i in range(args.serve_requests):
        if args.serve_config == "c4":
            inst = datagen.serving_instance(rng, seed=1000 + i)
        else:
            n = int(rng.integers(500, 2001))
            p = int(rng.integers(1000, 4001))
            inst = datagen.make_instance(n, p, corr="toeplitz", rho=float(rng.uniform(0, 0.7)),
                                         k=int(rng.integers(5, 13)), snr=float(rng.uniform(2, 10)),
                                         lambda0=0.005, lambda2=0.01, seed=1000 + i)
        reqs.append(inst)
        if (i + 1) % 8 == 0:
            print(json.dumps({"generated": i + 1, "s": round(time.perf_counter() - t_gen, 1)}), file=sys.stderr,
                  flush=True)
    kw = dict(K=args.serve_K, tol_node=1e-6, max_iter=2000, max_iter_root=10000, time_limit_s=args.serve_limit)
    prec = args.serve_precision
    out = {"metric": "time-to-certified-optimum under serving", "unit": "s",
           "config": {"workload": args.serve_config, "requests": len(reqs), "precision": prec, "K": args.serve_K,
                      "per_request_limit_s": args.serve_limit, "max_concurrent": args.serve_concurrent,
                      "hbm_budget": "80 % of free device memory"}}
    # solo times of the first draws: the arrival rate
    solo = []
    if args.serve_interarrival > 0:
        gap_mean = args.serve_interarrival
    else:
        srv = Server(0, hbm_budget_bytes=0, max_concurrent=1, **kw)
        for inst in reqs[:args.serve_solo]:
            rid = srv.submit(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision=prec)
            r = srv.wait(rid)
            solo.append({"n": inst.n, "p": inst.p, "ttco": round(r["done_s"] - r["admit_s"], 3),
                         "status": r["status"], "nodes": r["nodes_solved"]})
            print(json.dumps({"solo": solo[-1]}), file=sys.stderr, flush=True)
        srv.close()
        gap_mean = 0.5 * float(np.mean([x["ttco"] for x in solo]))
    out["config"]["mean_interarrival_s"] = round(gap_mean, 4)
    out["solo"] = solo
    gaps = np.random.default_rng(1).exponential(gap_mean, size=len(reqs))
    modes = {"on": [True], "off": [False], "both": [True, False]}[args.serve_batching]
    out["runs"] = {}
    for batching in modes:
        srv = Server(0, hbm_budget_bytes=0, max_concurrent=args.serve_concurrent, batching=batching, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ids = []
        for k, (inst, g) in enumerate(zip(reqs, gaps)):
            time.sleep(float(g))
            ids.append(srv.submit(inst.X, inst.y, inst.lambda0, inst.lambda2, inst.M, precision=prec))
            print(json.dumps({"batching": batching, "submitted": k + 1, "n": inst.n, "p": inst.p,
                              "t": round(time.perf_counter() - t0, 2)}), file=sys.stderr, flush=True)
        res = []
        for k, rid in enumerate(ids):
            res.append(srv.wait(rid))
            print(json.dumps({"batching": batching, "done": k + 1, "status": res[-1]["status"],
                              "ttco": round(res[-1]["done_s"] - res[-1]["submit_s"], 3)}), file=sys.stderr,
                  flush=True)
        wall = time.perf_counter() - t0
        st = srv.batching_stats()
        srv.close()
        tt = np.array([r["done_s"] - r["submit_s"] for r in res])
        wait = np.array([r["admit_s"] - r["submit_s"] for r in res])
        censored = [i for i, r in enumerate(res) if r["status"] != 0]
        nodes = sum(r["nodes_solved"] for r in res)
        out["runs"]["batching_on" if batching else "batching_off"] = {
            "requests": len(res), "certified": len(res) - len(censored), "censored": len(censored),
            "ttco_p50": round(float(np.percentile(tt, 50)), 4), "ttco_p99": round(float(np.percentile(tt, 99)), 4),
            "ttco_mean": round(float(tt.mean()), 4), "admit_wait_p50": round(float(np.percentile(wait, 50)), 4),
            "throughput_requests_per_s": round(len(res) / wall, 4), "node_relaxations_per_s": round(nodes / wall, 1),
            "wall_s": round(wall, 3), "executor": st,
            "instances_per_shared_launch": round(st["members"] / st["launches"], 3) if st["launches"] else None,
            "per_request": [{"n": i.n, "p": i.p, "ttco": round(float(t), 4), "nodes": r["nodes_solved"],
                             "status": r["status"], "peak_gb": round(r["peak_bytes"] / 1e9, 3)}
                            for i, t, r in zip(reqs, tt, res)]}
    print(json.dumps(out), flush=True)


def _serve_oracle_one(args):
    import oracle
    i, inst, max_nodes = args
    t0 = time.perf_counter()
    r = oracle.Oracle.from_instance(inst).bnb(tol_node=1e-6, max_iter=2000, max_iter_root=10000,
                                               max_nodes=max_nodes, trace_cap=0)
    return {"draw": i, "n": inst.n, "p": inst.p, "seconds": round(time.perf_counter() - t0, 2),
            "status": int(r["status"]), "nodes": int(r["nodes_solved"]), "certified": r["certified"],
            "support": [int(j) for j in r["support"]]}


def serve_oracle_main(args):
    """CPU baseline of the serving stream: the single-threaded oracle's branch
    and bound on the smallest draws (by n p) of the 64-instance stream, one
    process per instance, with a node cap (a capped run is censored)."""
    import multiprocessing as mp
    from paper_2602_04551_amd import datagen
    rng = np.random.default_rng(0)
    small = []
    for i in range(args.serve_requests):
        inst = datagen.serving_instance(rng, seed=1000 + i)
        small = sorted(small + [(i, inst)], key=lambda d: d[1].n * d[1].p)[:args.serve_oracle_count]
    workers = max(1, min(len(small), os.cpu_count() or 1, 16))
    rows = []
    with mp.get_context("fork").Pool(workers) as pool:
        for row in pool.imap_unordered(_serve_oracle_one, [(i, inst, args.serve_oracle_nodes) for i, inst in small]):
            rows.append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
    rows.sort(key=lambda r: r["draw"])
    out = {"metric": "CPU oracle time to certified optimum, smallest draws of the serving stream",
           "config": {"draws": args.serve_requests, "smallest": len(small), "node_cap": args.serve_oracle_nodes,
                      "workers": workers, "cpu_model": cpu_model()}, "runs": rows}
    print(json.dumps(out), flush=True)


def copy_bandwidth(nbytes=2 << 30, reps=5):
    """Device-to-device copy rate measured here (read + write bytes per second,
    best of `reps`), beside the 8 TB/s published HBM peak the rooflines use."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1.0)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del src, dst
    torch.cuda.empty_cache()
    gbs = 2 * nbytes / best / 1e9
    return {"GB_per_s": round(gbs, 1), "fraction_of_8000": round(gbs / 8000.0, 3),
            "what": f"{nbytes >> 20} MiB device copy, read plus write bytes over the best of {reps} event-timed copies"}


def main():
    args = parse()
    if args.traffic_summary:
        return traffic_summary(args.traffic_summary[0], args.traffic_summary[1], args.traffic_workload,
                               families=args.traffic_families.split(",") if args.traffic_families else None)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on exactly one GPU (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.batching:
        return batching_main(args)
    if args.highdim:
        return highdim_main(args)
    if args.serve:
        return serve_main(args)
    if args.node_parallel:
        return node_parallel_main(args)
    if args.heuristic_study:
        return heuristic_main(args)
    if args.serve_oracle:
        return serve_oracle_main(args)
    import torch
    from paper_2602_04551_amd import datagen

    if args.copy_calibrate:
        src = torch.empty(32 * 2**20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cfg, wl = HEADLINE
    inst = datagen.config_instance(cfg, seed=0)
    n, p, K = inst.n, inst.p, args.K
    codes = datagen.node_batch_codes(p, K, seed=K)
    root = fp64_root(inst)
    print(json.dumps({"root_sweeps": root[3], "root_ub": root[2]}), file=sys.stderr, flush=True)
    mixed = Path(inst, "bf16", codes, root)
    mixed.ctx.set_bf16_tile_rows(args.bf16_rows)
    dt, its, prof = run_path(mixed, args.steps, args.warmup)
    ms_per_step = 1e3 * dt / args.steps
    value = K * args.steps / dt
    roof, kernels = roofline(prof, n, p, workload=cfg.lower())
    out = {"metric": METRIC, "value": round(value, 2), "unit": "node relaxations/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic",
           "config": {"workload": wl.format(K=K), "n": n, "p": p, "K": K, "node_tol": 1e-6, "check_every": 10,
                      "rho": 1.0, "root_warm_start": f"FP64 root relaxation to a 1e-9 gap ({root[3]} sweeps), "
                                                     "shared by every precision",
                      "b_update": b_update_info(mixed.ctx), "bf16_tile_rows": args.bf16_rows},
           "roofline": roof,
           "roofline_hbm": sweep_bytes_roofline(prof, n, p, "bf16"),
           "kernels": kernels,
           "batch_detail": batch_detail(mixed),
           "set_data_s": {"bf16": round(mixed.set_data_s, 4)}}
    held, peak = mixed.ctx.memory_stats()
    out["hbm_high_water_gb"] = {"bf16": round(peak / 1e9, 3)}
    mixed.close()
    out["hbm_copy_measured"] = copy_bandwidth()
    print(json.dumps({"bf16": out["value"]}), file=sys.stderr, flush=True)
    if not args.only_mixed:
        for prec, steps_o in (("fp32", max(2, args.steps // 2)), ("fp64", max(2, args.steps // 4))):
            path = Path(inst, prec, codes, root)
            dt_o, _, prof_o = run_path(path, steps_o, 1)
            roof_o, kernels_o = roofline(prof_o, n, p)
            out[prec + "_path"] = {"value": round(K * steps_o / dt_o, 2), "unit": "node relaxations/s",
                                   "steps": steps_o, "ms_per_step": round(1e3 * dt_o / steps_o, 3),
                                   "roofline": roof_o, "kernels": kernels_o, "batch_detail": batch_detail(path),
                                   "b_update": b_update_info(path.ctx)}
            out["set_data_s"][prec] = round(path.set_data_s, 4)
            out["hbm_high_water_gb"][prec] = round(path.ctx.memory_stats()[1] / 1e9, 3)
            path.close()
            print(json.dumps({prec: out[prec + "_path"]["value"]}), file=sys.stderr, flush=True)
        out["mixed_vs_fp64"] = round(out["value"] / out["fp64_path"]["value"], 3)

    if not args.no_ttco:
        # time to certified optimum of the whole branch and bound, n = p = 1000, every precision
        from paper_2602_04551_amd.binding import Context
        inst2 = datagen.config_instance("C2", seed=0)
        tt = {}
        for prec in ("bf16", "fp32", "fp64", "fp8"):
            ctx = Context(0)
            t0 = time.perf_counter()
            ctx.set_data(inst2.X, inst2.y, inst2.lambda0, inst2.lambda2, inst2.M, precision=prec)
            torch.cuda.synchronize()
            sd = time.perf_counter() - t0
            ctx.bnb_solve(K=256, policy="best", tol_node=1e-6, max_iter=2000, max_iter_root=10000)   # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ctx.bnb_solve(K=256, policy="best", tol_node=1e-6, max_iter=2000, max_iter_root=10000)
            torch.cuda.synchronize()
            tt[prec] = {"seconds": round(time.perf_counter() - t0, 4), "set_data_s": round(sd, 4),
                        "nodes": r["nodes_solved"], "batches": r["batches"], "certified": r["certified"],
                        "lb": r["lb"], "status": r["status"], "support": [int(s) for s in r["support"]]}
            if prec in ("bf16", "fp64"):
                # the same solve with the matching-pursuit incumbent seeded before the root
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rh = ctx.bnb_solve(K=256, policy="best", tol_node=1e-6, max_iter=2000, max_iter_root=10000,
                                   root_heuristic=True)
                torch.cuda.synchronize()
                tt[prec]["with_heuristic"] = {"seconds": round(time.perf_counter() - t0, 4),
                                              "nodes": rh["nodes_solved"], "certified": rh["certified"],
                                              "status": rh["status"],
                                              "same_support": [int(s) for s in rh["support"]] == tt[prec]["support"]}
            ctx.close()
        gold = os.path.join(ROOT, "tests", "golden", "fullsize_c2_bnb.json")
        oracle_ttco = None
        if os.path.exists(gold):
            with open(gold) as f:
                g = json.load(f)
            oracle_ttco = {"seconds": g.get("cpu_seconds"), "nodes": g.get("nodes_solved"),
                           "what": "the single-threaded CPU oracle's depth-first branch and bound (K = 1) to "
                                   "certification on the same instance, timed when it wrote "
                                   "tests/golden/fullsize_c2_bnb.json (another host), same certified support"}
        out["ttco_n1000"] = {"workload": "n=p=1000 Toeplitz rho=0.5 k=10 SNR=5 lambda0=0.005 lambda2=0.01, "
                                         "best-first branch and bound with batches of 256 to certification "
                                         "(gap 0, eps_prune 2e-6), after one untimed solve",
                             "runs": tt, "oracle_cpu": oracle_ttco,
                             "mixed_vs_fp64": round(tt["fp64"]["seconds"] / tt["bf16"]["seconds"], 3)}
        print(json.dumps({"ttco": {k: v["seconds"] for k, v in tt.items()}}), file=sys.stderr, flush=True)
    if not args.no_highdim:
        inst5 = datagen.config_instance("C5", seed=0)
        root5 = fp64_root(inst5)
        runs = {prec: node_batch_run(inst5, prec, 1024, root5) for prec in ("fp8", "bf16", "fp32", "fp64")}
        queue = {prec: node_queue_run(inst5, prec, 4096, 1024, root5) for prec in ("fp8", "fp64")}
        out["highdim_n1000_p50000"] = {
            "workload": "n=1000 p=50000 constant correlation 0.2 k=25 SNR=3 lambda0=0.002 lambda2=0.005, node "
                        "batches of 1024 (free sets U{50..p}, |F1| U{0..20}) from the FP64 root",
            "runs": runs, "fp8_vs_fp64": round(runs["fp8"]["value"] / runs["fp64"]["value"], 3),
            "queue": {"what": "4096 queued nodes of the same workload through 1024 slots refilled as nodes "
                              "retire (continuous batching), against the fixed batch of 1024 above",
                      "runs": queue,
                      "fp8_queue_vs_batch": round(queue["fp8"]["value"] / runs["fp8"]["value"], 3)}}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, K, root, args.cpu_seconds, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
