"""Throughput benchmark of the patch-guided nested-dissection ordering.

One step = one full ordering (Alg. 1: patches, quotient graph, separator
tree, local minimum-degree orders, concatenation, elimination tree, column
counts) of a 1024x1024 torus triangle mesh (1,048,576 vertices, seeded
diagonals, scalar int32 CSR pattern + diagonal) with target patch size 512,
inputs resident in device memory before the timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

Prints one JSON line.  `value` is mesh vertices ordered per second (whole
job), `roofline` rates the dominant kernel against MI355X's HBM peak with
algorithmic bytes, `cpu_baseline` times the serial CPU oracle on one core
over a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

# 1024x1024 torus, seed 2, S = 512
H = W = 1024
MESH_SEED = 2
PATCH = 512


def kernel_bytes(name, n, nnz, P, D, lloyd):
    """Algorithmic bytes one launch of a dominant kernel must move (int32).

    Per-vertex figures: a CSR pass reads rowptr (4 B) and the row (4 B per
    entry); state arrays are read or written once at 4 B a vertex.
    """
    csr = 4 * (n + 1) + 4 * nnz
    if name == "local_orders":
        # gather every node's induced rows once (CSR + node_of + local index),
        # write the local order
        return csr + 4 * n * 3
    if name == "symbolic":
        # read the permuted pattern once (CSR + iperm + node_of), write parent
        # and colcount
        return csr + 4 * n * 4
    if name == "patches":
        # (1 + 2 * lloyd) growth passes over the CSR, plus labels
        return (1 + 2 * lloyd) * (csr + 8 * n)
    if name == "septree":
        # D levels over the CSR of boundary vertices (at most the whole CSR)
        return D * (csr + 8 * n)
    return csr + 8 * n


def run_gpu(args):
    import numpy as np  # noqa: F401
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    from paper_2602_00898_amd import meshgen as mg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    A = mg.grid_mesh(H, W, True, MESH_SEED)
    n, nnz = A.n, A.nnz
    rp = torch.from_numpy(A.rowptr).to(dev)
    ci = torch.from_numpy(A.colind).to(dev)
    h = fpm.Handle()
    opts = fpm.options(PATCH, fpm.SCHED_LEVEL, 1, 1, MESH_SEED, fpm.FLAG_TIMING)
    ws_bytes, max_nodes = fpm.query(h, n, rp, ci, opts)
    i32 = dict(dtype=torch.int32, device=dev)
    out = dict(perm=torch.empty(n, **i32), iperm=torch.empty(n, **i32),
               parent=torch.empty(n, **i32), colcount=torch.empty(n, **i32),
               nnzL=torch.zeros(1, dtype=torch.int64, device=dev),
               node_begin=torch.empty(max_nodes, **i32), node_size=torch.empty(max_nodes, **i32),
               gmap=torch.empty(n, **i32), n_nodes=torch.zeros(1, **i32),
               status=torch.zeros(1, dtype=torch.int32, device=dev))
    h.workspace(ws_bytes, dev)
    torch.cuda.synchronize(dev)

    def step():
        return fpm.order(rp, ci, n, patch_size=PATCH, seed=MESH_SEED, handle=h, out=out,
                         timing=True)

    for i in range(args.warmup):
        t = time.perf_counter()
        step()
        torch.cuda.synchronize(dev)
        print(f"[bench] warmup {i}: {1e3 * (time.perf_counter() - t):.2f} ms", file=sys.stderr, flush=True)
    stages = {}
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        for k, v in fpm.stage_times(h).items():
            stages.setdefault(k, []).append(v)
        if i % 5 == 0:
            print(f"[bench] step {i}", file=sys.stderr, flush=True)
    torch.cuda.synchronize(dev)
    dt = time.perf_counter() - t0
    nnzL = int(out["nnzL"].item())
    P = int(out["gmap"].max().item()) + 1
    nn = int(out["n_nodes"].item())
    D = max(0, (nn + 1).bit_length() - 2)
    mean_ms = {k: sum(v) / len(v) for k, v in stages.items()}
    dom = max(mean_ms, key=mean_ms.get)
    byts = kernel_bytes(dom, n, nnz, P, D, 1)
    achieved = byts / (mean_ms[dom] * 1e-3) / 1e9
    ms = dt * 1e3 / args.steps
    return dict(n=n, nnz=nnz, nnzL=nnzL, P=P, D=D, ms=ms, dt=dt, stage_ms=mean_ms, dom=dom,
                dom_bytes=byts, achieved=achieved, A=A)


def run_cpu(A, budget_s=15.0):
    import oracle

    oracle.build()
    print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
    times = []
    t_all = time.perf_counter()
    while True:
        t = time.perf_counter()
        r = oracle.order(A.rowptr, A.colind, A.n, patch_size=PATCH, seed=MESH_SEED)
        times.append(time.perf_counter() - t)
        if time.perf_counter() - t_all > budget_s or len(times) >= 5:
            break
    med = statistics.median(times)
    return dict(value=A.n / med / 1e6, unit="M vertices/s", cores=1, kind="oracle",
                sample=f"{len(times)} full orderings of the 1024x1024 torus (S=512) on one "
                       f"host core, median {med:.3f} s", nnzL=r["nnzL"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the ordering of one mesh is not sharded across "
              "GPUs in this library (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    g = run_gpu(args)
    cpu = None if args.no_cpu else run_cpu(g["A"])
    if cpu is not None and cpu.pop("nnzL") != g["nnzL"]:
        print(f"nnz(L) differs from the oracle: {g['nnzL']} vs oracle", file=sys.stderr)
        sys.exit(1)
    line = {
        "metric": "M mesh vertices permuted/s",
        "value": round(g["n"] / (g["ms"] * 1e-3) / 1e6, 4),
        "unit": "M vertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(g["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "1024x1024 torus triangle mesh, seeded diagonals, S=512",
                   "n": g["n"], "nnz": g["nnz"], "patch_size": PATCH, "patches": g["P"],
                   "depth": g["D"], "nnzL": g["nnzL"]},
        "roofline": {"bound": "hbm", "kernel": g["dom"], "achieved": round(g["achieved"], 3),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(g["achieved"] / HBM_PEAK_GBS, 6), "traffic": None,
                     "bytes_per_launch": g["dom_bytes"],
                     "launch_ms": round(g["stage_ms"][g["dom"]], 4)},
        "stage_ms": {k: round(v, 4) for k, v in g["stage_ms"].items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
