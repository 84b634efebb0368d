"""Throughput benchmark of the patch-guided nested-dissection ordering.

One step = one full ordering (Alg. 1: patches, quotient graph, separator
tree, local minimum-degree orders, concatenation, elimination tree, column
counts) of a 1024x1024 torus triangle mesh (1,048,576 vertices, seeded
diagonals, scalar int32 CSR pattern + diagonal) with target patch size 512,
inputs resident in device memory before the timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-batch]
                    [--no-serve] [--no-update] [--no-block] [--serve-requests R]
                    [--slots L] [--copy-probe-mib M]
    python bench.py --traffic-from FETCH.csv WRITE.csv [--copy-probe-mib M]

Prints one JSON line.  `value` is mesh vertices ordered per second (whole
job).  `roofline` rates the dominant kernel (the largest event-timed total
per ordering; its launches timed with HIP events on their own streams during
the timed steps) against MI355X's HBM peak with the algorithmic bytes of the
path's byte budget; its `traffic` is the HBM bytes per launch that two
rocprofv3 counter runs measured (FETCH_SIZE, WRITE_SIZE, each scaled by what
the counter reads for a plain device copy of known size), kept in
profiles/traffic.json with a digest of the kernel sources and reported only
while the sources still match.  `path_roofline` rates the whole path the
same way, `kernels` every timed kernel.  `cpu_baseline` times the serial CPU
oracle on one host core over a bounded sample (and the 256-mesh batch with
one process per core).  `batch` compares ordering 256 meshes of uneven size
one at a time with the batched call, `serving` drives the request server
with Poisson arrivals and reports p50/p99 latency, `update` re-orders the
benchmark mesh after a local pattern change, `block` orders the 2048x2048
torus in 3x3 blocks.
"""

from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics
import sys
import time

# The served run keeps 16 slots (streams) busy; HIP maps streams onto
# GPU_MAX_HW_QUEUES hardware queues (4 by default, which serialises the
# slots), so raise it to 16 before anything initialises HIP.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < 16:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

# 1024x1024 torus, seed 2, S = 512
H = W = 1024
MESH_SEED = 2
PATCH = 512
# kernels timed one by one with HIP events during the warm-up orderings
KERNELS = ("k_md_top", "k_md", "k_sym_elim", "k_sym_prep", "k_bfs_level", "k_bisect")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def csrc_digest():
    """sha256 over the HIP sources (names and contents) of the library."""
    d = os.path.join(ROOT, "paper_2602_00898_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


def traffic_for(kernel):
    """Measured HBM bytes per launch of a kernel, or None when there is no
    measurement for the current sources."""
    try:
        with open(TRAFFIC) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("csrc_sha256") != csrc_digest():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k["bytes_per_launch"]


def copy_probe(mib):
    """A plain device copy of known size, for calibrating the byte counters
    (an elementwise kernel rather than a DMA copy, so the counters see it)."""
    import torch
    dev = torch.device("cuda:0")
    src = torch.ones(mib << 18, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1, out=dst)  # an elementwise kernel: reads and writes mib MiB
    torch.cuda.synchronize(dev)
    log(f"copy probe: 3 x {mib} MiB")


def _counter_rows(path, counter):
    """(kernel name, value) of every dispatch row of one counter."""
    out = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") == counter:
                out.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return out


def traffic_from(fetch_csv, write_csv, mib):
    """Write profiles/traffic.json from a FETCH_SIZE run and a WRITE_SIZE run
    of `bench.py --copy-probe-mib M` (counter values in KiB per dispatch)."""
    known = float(mib << 20)
    res = {}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = _counter_rows(path, counter)
        cp = [v * 1024.0 for k, v in rows if "copy" in k.lower() or "elementwise" in k.lower()]
        cp = [v for v in cp if v > 0.5 * known]
        if not cp:
            raise SystemExit(f"no copy-probe dispatch in {path}")
        factor = known / statistics.median(cp)
        per = {}
        for k, v in rows:
            name = k.split("(")[0].strip()
            if name in KERNELS:
                per.setdefault(name, []).append(v * 1024.0 * factor)
        res[key] = (factor, per)
    kernels = {}
    for name in set(res["fetch"][1]) & set(res["write"][1]):
        f, w = res["fetch"][1][name], res["write"][1][name]
        kernels[name] = {"fetch_bytes_per_launch": round(sum(f) / len(f)),
                         "write_bytes_per_launch": round(sum(w) / len(w)),
                         "bytes_per_launch": round(sum(f) / len(f) + sum(w) / len(w)),
                         "launches": len(f)}
    out = {"csrc_sha256": csrc_digest(), "copy_probe_mib": mib,
           "fetch_factor": round(res["fetch"][0], 4), "write_factor": round(res["write"][0], 4),
           "kernels": kernels}
    with open(TRAFFIC, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def csr_pass_bytes(n, nnz):
    """One pass over the CSR pattern per vertex: 4 B of row pointer plus 4 B
    per stored entry (diagonal included): 32 B on a torus (7 entries)."""
    return 4.0 + 4.0 * nnz / max(n, 1)


def kernel_bytes(name, n, nnz, top_vertices, lloyd_iters=1):
    """Algorithmic HBM bytes of all launches of a kernel in one ordering, by
    the per-vertex figures of the path's byte budget (c = one CSR pass):
    patching takes (1 + 2 I) passes (the BFS launches), each local order
    gathers its node's rows once (one pass over the vertices it orders),
    the symbolic stage reads the permuted pattern once plus 24 B of iperm
    gathers and writes parent and column count (8 B).  The bisection works
    on the quotient graph only (no per-vertex bytes)."""
    c = csr_pass_bytes(n, nnz)
    if name == "k_bfs_level":
        return (1 + 2 * lloyd_iters) * c * n
    if name == "k_md":
        return c * (n - top_vertices)
    if name == "k_md_top":
        return c * top_vertices
    if name == "k_sym_prep":
        return (c + 24.0) * n
    if name == "k_sym_elim":
        return 8.0 * n
    return 0.0


def path_bytes_per_vertex(n, nnz, depth, beta, lloyd_iters=1):
    """Algorithmic bytes per vertex of the whole path: (4 + 2 I) CSR passes
    (patching, boundary detection, local-order gather, symbolic), the marking
    passes over the boundary list (depth x beta passes, beta = boundary
    fraction), and 64 B of state arrays and outputs."""
    c = csr_pass_bytes(n, nnz)
    return (4 + 2 * lloyd_iters) * c + depth * beta * c + 64.0


def boundary_fraction(rowptr, colind, gmap):
    """Fraction of vertices with a neighbour in another patch."""
    import numpy as np
    rows = np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))
    g = np.asarray(gmap)
    cross = g[rows] != g[colind]
    return float(np.unique(rows[cross]).size) / max(len(rowptr) - 1, 1)


# ------------------------------------------------------------------ inputs
def make_inputs(args):
    """Generate every input before the GPU is touched (forked pool)."""
    import multiprocessing as mp

    from paper_2602_00898_amd import meshgen as mg
    from paper_2602_00898_amd import workloads as wl
    t = time.perf_counter()
    A = mg.grid_mesh(H, W, True, MESH_SEED)
    batch = serve = None
    procs = min(16, os.cpu_count() or 1)
    pool = mp.get_context("fork").Pool(procs)
    try:
        if not args.no_batch:
            batch = pool.map(wl.batch_mesh, wl.batch_specs(), chunksize=4)
        if not args.no_serve:
            stream = wl.serving_stream(args.serve_requests)
            meshes = pool.map(wl.serving_mesh, [s for _, s in stream], chunksize=2)
            serve = [(t_arr, m) for (t_arr, _), m in zip(stream, meshes)]
    finally:
        # close and join (not terminate): the workers exit on their own, so a
        # profiled run sees no signal
        pool.close()
        pool.join()
    log(f"inputs generated in {time.perf_counter() - t:.1f} s with {procs} processes")
    return A, batch, serve


# ------------------------------------------------------------------ plain
def run_plain(args, A):
    import torch

    from paper_2602_00898_amd import fastperm as fpm

    dev = torch.device("cuda:0")
    n, nnz = A.n, A.nnz
    rp = torch.from_numpy(A.rowptr).to(dev)
    ci = torch.from_numpy(A.colind).to(dev)
    from paper_2602_00898_amd import autotune
    h = fpm.Handle()
    autotune.apply(h, autotune.exec_for(n))  # execution settings only: same result
    opts = fpm.options(PATCH, fpm.SCHED_LEVEL, 1, 1, MESH_SEED, fpm.FLAG_TIMING)
    ws_bytes, max_nodes = fpm.query(h, n, rp, ci, opts)
    out = fpm._alloc_out(n, max_nodes, 1, dev)
    h.workspace(ws_bytes, dev)
    torch.cuda.synchronize(dev)

    def step():
        return fpm.order(rp, ci, n, patch_size=PATCH, seed=MESH_SEED, handle=h, out=out,
                         timing=True)

    # warmup; the first warmups also time the candidate kernels one by one
    # (HIP events around each launch, on the launch's own stream)
    timed = {}
    for i in range(max(args.warmup, len(KERNELS))):
        cand = KERNELS[i] if i < len(KERNELS) else None
        fpm.time_kernel(h, cand)
        t = time.perf_counter()
        step()
        torch.cuda.synchronize(dev)
        if cand:
            timed[cand] = fpm.kernel_time(h)
        log(f"warmup {i}: {1e3 * (time.perf_counter() - t):.2f} ms")
    # the dominant kernel: the largest event-timed total per ordering
    dom = max(timed, key=lambda k: timed[k][0])
    fpm.time_kernel(h, dom)
    stages = {}
    kt_ms, kt_launch = 0.0, 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        for k, v in fpm.stage_times(h).items():
            stages.setdefault(k, []).append(v)
        ms, nl = fpm.kernel_time(h)
        kt_ms += ms
        kt_launch += nl
        if i % 5 == 0:
            log(f"step {i}")
    torch.cuda.synchronize(dev)
    dt = time.perf_counter() - t0
    fpm.time_kernel(h, None)
    nnzL = int(out["nnzL"].item())
    gmap = out["gmap"][:n].cpu().numpy()
    P = int(gmap.max()) + 1
    nn = int(out["n_nodes"].item())
    D = max(0, (nn + 1).bit_length() - 2)
    sizes = out["node_size"][:nn].cpu().numpy()
    top_vertices = int(sizes[:min(nn, 7)].sum())  # separators of depths 0-2
    beta = boundary_fraction(A.rowptr, A.colind, gmap)
    kern = {}
    for k, (ms, nl) in timed.items():
        alg = kernel_bytes(k, n, nnz, top_vertices)
        per = alg / max(nl, 1)
        avg = ms / max(nl, 1)
        gbs = per / (avg * 1e-3) / 1e9 if avg > 0 else 0.0
        kern[k] = {"ms_per_ordering": round(ms, 4), "launches": nl, "avg_launch_ms": round(avg, 5),
                   "alg_bytes_per_launch": round(per), "GBps": round(gbs, 4),
                   "frac": round(gbs / HBM_PEAK_GBS, 7)}
    per_launch_bytes = kernel_bytes(dom, n, nnz, top_vertices) * args.steps / max(kt_launch, 1)
    avg_ms = kt_ms / max(kt_launch, 1)
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    return dict(n=n, nnz=nnz, nnzL=nnzL, P=P, D=D, ms=dt * 1e3 / args.steps, tuning=h.tuning()[:2],
                stage_ms={k: sum(v) / len(v) for k, v in stages.items()}, dom=dom,
                dom_bytes=per_launch_bytes, dom_avg_ms=avg_ms, dom_launches=kt_launch / args.steps,
                achieved=achieved, kernels=kern, beta=beta,
                path_bpv=path_bytes_per_vertex(n, nnz, D, beta))


# ------------------------------------------------------------------ batch
def run_batch(args, meshes):
    import torch

    from paper_2602_00898_amd import fastperm as fpm

    dev = torch.device("cuda:0")
    from paper_2602_00898_amd import workloads as wl
    dm = [dict(rowptr=torch.from_numpy(A.rowptr).to(dev), colind=torch.from_numpy(A.colind).to(dev),
               n=A.n, patch_size=wl.batch_patch_size(A.n), seed=wl.batch_order_seed(i))
          for i, A in enumerate(meshes)]
    nv = sum(A.n for A in meshes)
    h = fpm.Handle()
    torch.cuda.synchronize(dev)
    # plain: one call per mesh, one stream, queued back to back on outputs
    # allocated by a first pass (as the batch below)
    plain_out = [fpm.order(m["rowptr"], m["colind"], m["n"], patch_size=m["patch_size"],
                           seed=m["seed"], handle=h) for m in dm]
    torch.cuda.synchronize(dev)
    t = time.perf_counter()
    for m, o in zip(dm, plain_out):
        fpm.order(m["rowptr"], m["colind"], m["n"], patch_size=m["patch_size"], seed=m["seed"],
                  handle=h, out=o, check=False)
    torch.cuda.synchronize(dev)
    t_plain = time.perf_counter() - t
    if any(int(o["status"].item()) for o in plain_out):
        raise SystemExit("batch plain: device error bits set")
    log(f"batch plain: {t_plain:.2f} s")
    from paper_2602_00898_amd import autotune
    hb = fpm.Handle()
    autotune.apply(hb, autotune.exec_batch())
    bout = fpm.order_batch(dm, handle=hb)  # warm-up; allocates the outputs
    torch.cuda.synchronize(dev)
    reps = 3
    t = time.perf_counter()
    for _ in range(reps):
        bout = fpm.order_batch(dm, handle=hb, outs=bout, check=False)
    torch.cuda.synchronize(dev)
    t_batch = (time.perf_counter() - t) / reps
    if any(int(o["status"].item()) for o in bout):
        raise SystemExit("batch: device error bits set")
    log(f"batch batched: {t_batch:.3f} s")
    # the same batch recorded once into a HIP graph, then replayed
    gb = fpm.Graph(dm, handle=hb)
    gb.launch()
    torch.cuda.synchronize(dev)
    reps = 3
    t = time.perf_counter()
    for _ in range(reps):
        gout = gb.launch()
    torch.cuda.synchronize(dev)
    t_graph = (time.perf_counter() - t) / reps
    log(f"batch graph replay: {t_graph:.3f} s")
    same = all(torch.equal(a[k], b[k]) and torch.equal(a[k], c[k])
               for a, b, c in zip(plain_out, bout, gout)
               for k in ("perm", "iperm", "parent", "colcount", "nnzL"))
    del gb
    return {"workload": "256 grid/torus meshes, sides log-uniform 45..447, 5% edge flips, "
                        "S from the autotune table",
            "meshes": len(meshes), "vertices": nv,
            "plain_value": round(nv / t_plain / 1e6, 4), "batched_value": round(nv / t_batch / 1e6, 4),
            "graph_replay_value": round(nv / t_graph / 1e6, 4),
            "unit": "M vertices/s", "speedup": round(t_plain / t_batch, 3),
            "tuning": list(hb.tuning()[:2]),
            "identical_to_plain": bool(same)}


# ------------------------------------------------------------------ graph
def run_graph(args):
    """Latency of one small mesh: a call per ordering against the replay of
    a recorded graph (no host work between the stages either way; the graph
    also saves the host's per-launch cost)."""
    import torch

    from paper_2602_00898_amd import autotune
    from paper_2602_00898_amd import fastperm as fpm
    from paper_2602_00898_amd import meshgen as mg

    dev = torch.device("cuda:0")
    res = {}
    for side in (64, 256):
        A = mg.grid_mesh(side, side, True, MESH_SEED, 0.05)
        rp = torch.from_numpy(A.rowptr).to(dev)
        ci = torch.from_numpy(A.colind).to(dev)
        S = autotune.patch_size_for(A.n)
        h = fpm.Handle()
        autotune.apply(h, autotune.exec_for(A.n))
        opts = fpm.options(S, fpm.SCHED_LEVEL, 1, 1, MESH_SEED)
        ws_bytes, max_nodes = fpm.query(h, A.n, rp, ci, opts)
        out = fpm._alloc_out(A.n, max_nodes, 1, dev)
        h.workspace(ws_bytes, dev)

        def eager():
            fpm.order(rp, ci, A.n, patch_size=S, seed=MESH_SEED, handle=h, out=out, check=False)

        g = fpm.Graph([dict(rowptr=rp, colind=ci, n=A.n, patch_size=S, seed=MESH_SEED)], handle=h)
        # latency of one ordering (synchronised after each call): the median
        # of 25 calls, in three alternating rounds, the best round kept
        times = {"eager": float("inf"), "graph": float("inf")}
        for _ in range(3):
            for name, fn in (("eager", eager), ("graph", g.launch)):
                for _ in range(3):
                    fn()
                torch.cuda.synchronize(dev)
                ts = []
                for _ in range(25):
                    t = time.perf_counter()
                    fn()
                    torch.cuda.synchronize(dev)
                    ts.append(time.perf_counter() - t)
                times[name] = min(times[name], sorted(ts)[len(ts) // 2] * 1e3)
        same = all(torch.equal(out[k], g.outputs[0][k]) for k in ("perm", "parent", "colcount"))
        res[f"torus{side}x{side}"] = {"n": A.n, "patch_size": S,
                                      "eager_ms": round(times["eager"], 4),
                                      "graph_ms": round(times["graph"], 4),
                                      "identical": bool(same)}
        log(f"graph {side}x{side}: eager {times['eager']:.3f} ms, graph {times['graph']:.3f} ms")
        del g
    return res


# ------------------------------------------------------------------ fill
FILL_S = (64, 128, 256, 512, 1024)
FILL_MODES = (("one-sided, full depth", -1, False), ("refined, full depth", -1, True),
              ("refined, nd_level 10", 10, True), ("refined, AMD", -1, "amd"))


def run_fill(args):
    """Ordering quality against the patch size: nnz(L)/nnz(A) (A with its
    diagonal) and the ordering time for S in FILL_S, for the separator modes
    of FILL_MODES, on a 548x548 torus (300K vertices) and the 1024x1024 one."""
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    from paper_2602_00898_amd import meshgen as mg

    dev = torch.device("cuda:0")
    res = []
    for side in (548, 1024):
        A = mg.grid_mesh(side, side, True, MESH_SEED, 0.05)
        rp = torch.from_numpy(A.rowptr).to(dev)
        ci = torch.from_numpy(A.colind).to(dev)
        nnzA = A.nnz  # the pattern includes the diagonal
        h = fpm.Handle()
        for label, L, ref in FILL_MODES:
            row = {"mesh": f"torus {side}x{side}", "n": A.n, "mode": label, "fill": {}, "ms": {}}
            for S in FILL_S:
                def run():
                    return fpm.order(rp, ci, A.n, patch_size=S, seed=MESH_SEED, handle=h,
                                     nd_level=L, refine=bool(ref), amd=ref == "amd")
                run()
                torch.cuda.synchronize(dev)
                t = time.perf_counter()
                out = run()
                torch.cuda.synchronize(dev)
                row["ms"][S] = round((time.perf_counter() - t) * 1e3, 3)
                row["fill"][S] = round(int(out["nnzL"].item()) / nnzA, 4)
            log(f"fill {side}x{side} {label}: {row['fill']}")
            res.append(row)
    return {"metric": "nnz(L)/nnz(A)", "patch_sizes": list(FILL_S), "rows": res}


# ------------------------------------------------------------------ modes
MODES = (("exact MD, one-sided separators (default)", dict()),
         ("exact MD, refined separators", dict(refine=True)),
         ("AMD, one-sided separators", dict(amd=True)),
         ("AMD, refined separators", dict(amd=True, refine=True)),
         ("AMD, refined, nd_level 10", dict(amd=True, refine=True, nd_level=10)))


def run_modes(args, A):
    """The headline mesh under each separator / local-order mode: time per
    ordering as the headline measures it (8 orderings queued back to back on
    preallocated outputs, then one synchronisation) and nnz(L)/nnz(A)."""
    import torch

    from paper_2602_00898_amd import autotune
    from paper_2602_00898_amd import fastperm as fpm

    dev = torch.device("cuda:0")
    rp = torch.from_numpy(A.rowptr).to(dev)
    ci = torch.from_numpy(A.colind).to(dev)
    h = fpm.Handle()
    autotune.apply(h, autotune.exec_for(A.n))
    res = []
    for label, kw in MODES:
        out = fpm.order(rp, ci, A.n, patch_size=PATCH, seed=MESH_SEED, handle=h, **kw)
        torch.cuda.synchronize(dev)

        def run():
            fpm.order(rp, ci, A.n, patch_size=PATCH, seed=MESH_SEED, handle=h, out=out,
                      check=False, **kw)
        run()
        torch.cuda.synchronize(dev)
        reps = 8
        t = time.perf_counter()
        for _ in range(reps):
            run()
        torch.cuda.synchronize(dev)
        ms = (time.perf_counter() - t) / reps * 1e3
        if int(out["status"].item()) != 0:
            raise SystemExit(f"mode {label}: device error bits {int(out['status'].item()):#x}")
        res.append({"mode": label, "ms": round(ms, 3),
                    "value": round(A.n / (ms * 1e-3) / 1e6, 3),
                    "fill": round(int(out["nnzL"].item()) / A.nnz, 4)})
        log(f"mode {label}: {ms:.2f} ms, fill {res[-1]['fill']}")
    return {"workload": "1024x1024 torus, S=512", "unit": "M vertices/s", "rows": res}


# ------------------------------------------------------------------ update
def run_update(args, A):
    """Pattern change on the benchmark mesh: 16 quads in one corner get their
    other diagonal; the new pattern is ordered again with the earlier call's
    patches kept (fp_order_update), reusing the local orders of unchanged
    nodes, against a full ordering of the new pattern with the same patches."""
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    from paper_2602_00898_amd import meshgen as mg

    dev = torch.device("cuda:0")
    quads = [(100 + i, 100 + j) for i in range(4) for j in range(4)]
    B = mg.swap_quad_diagonals(A, W, quads)
    rp, ci = torch.from_numpy(A.rowptr).to(dev), torch.from_numpy(A.colind).to(dev)
    rp2, ci2 = torch.from_numpy(B.rowptr).to(dev), torch.from_numpy(B.colind).to(dev)
    h0, h1, h2 = fpm.Handle(), fpm.Handle(), fpm.Handle()
    first = fpm.order(rp, ci, A.n, patch_size=PATCH, seed=MESH_SEED, handle=h0)
    gmap = first["gmap"][:A.n].clone()
    steps = max(1, min(args.steps, 10))

    def timed(fn):
        for _ in range(2):
            out = fn()
        torch.cuda.synchronize(dev)
        t = time.perf_counter()
        for _ in range(steps):
            out = fn()
        torch.cuda.synchronize(dev)
        return out, (time.perf_counter() - t) * 1e3 / steps

    upd, ms_u = timed(lambda: fpm.order_update(rp2, ci2, B.n, gmap, h0._ws, patch_size=PATCH,
                                               seed=MESH_SEED, handle=h1))
    full, ms_f = timed(lambda: fpm.order(rp2, ci2, B.n, patch_size=PATCH, user_gmap=gmap,
                                         handle=h2))
    same = all(torch.equal(upd[k], full[k]) for k in ("perm", "iperm", "parent", "colcount", "nnzL"))
    reused = int(upd["reused"].item())
    return {"workload": "1024x1024 torus, S=512, 16 quads in one corner flipped to the other "
                        "diagonal, patches of the earlier ordering kept",
            "steps": steps, "ms_update": round(ms_u, 3), "ms_full": round(ms_f, 3),
            "speedup": round(ms_f / ms_u, 3), "reused_fraction": round(reused / A.n, 5),
            "identical_to_full": bool(same)}


# ------------------------------------------------------------------ block
BLOCK_SIDE, BLOCK_SEED, BLOCK_B = 2048, 4, 3


def run_block(args):
    """2048x2048 torus expanded to dense 3x3 blocks (12.6M DOF, 264M entries,
    int64 row pointers), ordered on the vertex graph and expanded back."""
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    from paper_2602_00898_amd import meshgen as mg

    t = time.perf_counter()
    A = mg.grid_mesh(BLOCK_SIDE, BLOCK_SIDE, True, BLOCK_SEED)
    B = mg.block_expand(A, BLOCK_B)
    log(f"block pattern generated in {time.perf_counter() - t:.1f} s")
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(B.rowptr).to(dev)
    ci = torch.from_numpy(B.colind).to(dev)
    del B
    h = fpm.Handle()

    def step():
        return fpm.order(rp, ci, rp.numel() - 1, patch_size=PATCH, seed=BLOCK_SEED,
                         block_size=BLOCK_B, handle=h)

    for _ in range(2):
        out = step()
    torch.cuda.synchronize(dev)
    steps = max(1, min(args.steps, 5))
    t = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize(dev)
    ms = (time.perf_counter() - t) * 1e3 / steps
    return {"workload": "2048x2048 torus, seeded diagonals, dense 3x3 blocks, int64 row pointers, S=512",
            "vertices": A.n, "dof": A.n * BLOCK_B, "nnz": int(ci.numel()), "steps": steps,
            "ms_per_ordering": round(ms, 3), "value": round(A.n / ms / 1e3, 4),
            "dof_per_s_M": round(A.n * BLOCK_B / ms / 1e3, 4), "unit": "M vertices/s",
            "nnzL": int(out["nnzL"].item())}


# ------------------------------------------------------------------ serving
def run_serve(args, reqs):
    from paper_2602_00898_amd import fastperm as fpm
    from paper_2602_00898_amd import workloads as wl

    srv = fpm.Server(hbm_budget=args.serve_budget_gb << 30, max_slots=args.slots)
    try:
        # warm the slots on a small request
        A0 = reqs[0][1]
        srv.wait(srv.submit(A0.rowptr, A0.colind, A0.n, patch_size=PATCH, seed=1))
        t0 = time.perf_counter()
        tickets = []
        for t_arr, A in reqs:  # open loop: submit at the arrival time
            delay = t0 + t_arr - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets.append(srv.submit(A.rowptr, A.colind, A.n, patch_size=wl.SERVE_PATCH,
                                      seed=wl.SERVE_ORDER_SEED))
        lat = []
        for tk in tickets:
            lat.append(srv.wait(tk)["latency_s"])
        wall = time.perf_counter() - t0
    finally:
        srv.close()
    lat.sort()
    nv = sum(A.n for _, A in reqs)

    def pct(p):
        return lat[min(len(lat) - 1, int(round(p / 100.0 * (len(lat) - 1))))]

    return {"workload": f"Poisson arrivals {wl.SERVE_RATE:.0f}/s, grid/torus sides log-uniform "
                        "100..1414 (1e4..2e6 vertices), fresh diagonals per request, S=512",
            "requests": len(reqs), "vertices": nv, "slots": args.slots,
            "value": round(nv / wall / 1e6, 4), "unit": "M vertices/s",
            "p50_ms": round(1e3 * pct(50), 2), "p99_ms": round(1e3 * pct(99), 2),
            "offered_M_vertices_per_s": round(nv / reqs[-1][0] / 1e6, 2)}


# ------------------------------------------------------------------ oracle
def host_cpu():
    """Model name of the host CPU and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def _oracle_batch_item(args):
    import oracle
    A, S, seed = args
    t = time.perf_counter()
    oracle.order(A.rowptr, A.colind, A.n, patch_size=S, seed=seed)
    return time.perf_counter() - t


def run_cpu(A, batch_meshes, budget_s=15.0):
    """The oracle as it stands: full orderings of the benchmark mesh on one
    core (median), and the 256-mesh batch with one process per core."""
    import multiprocessing as mp

    import oracle
    from paper_2602_00898_amd import workloads as wl

    oracle.build()
    model, cores = host_cpu()
    log(f"CPU oracle baseline on {cores} cores of {model}")
    times = []
    t_all = time.perf_counter()
    while True:
        t = time.perf_counter()
        r = oracle.order(A.rowptr, A.colind, A.n, patch_size=PATCH, seed=MESH_SEED)
        times.append(time.perf_counter() - t)
        if time.perf_counter() - t_all > budget_s or len(times) >= 5:
            break
    med = statistics.median(times)
    res = dict(value=A.n / med / 1e6, unit="M vertices/s", cores=1, kind="oracle",
               host_cpu=model, host_cores=cores,
               sample=f"{len(times)} full orderings of the 1024x1024 torus (S=512) on one "
                      f"host core, median {med:.3f} s", nnzL=r["nnzL"])
    if batch_meshes is not None:
        items = [(M, wl.batch_patch_size(M.n), wl.batch_order_seed(i))
                 for i, M in enumerate(batch_meshes)]
        items.sort(key=lambda x: -x[0].n)
        t = time.perf_counter()
        pool = mp.get_context("fork").Pool(cores)
        try:
            pool.map(_oracle_batch_item, items, chunksize=1)
        finally:
            pool.close()
            pool.join()
        wall = time.perf_counter() - t
        nv = sum(M.n for M in batch_meshes)
        res["batch_all_cores"] = dict(value=round(nv / wall / 1e6, 4), unit="M vertices/s",
                                      processes=cores, meshes=len(batch_meshes),
                                      sample=f"the 256-mesh batch, one oracle process per core, "
                                             f"{wall:.2f} s wall")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-mesh batch")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving sample")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-budget-gb", type=int, default=64)
    ap.add_argument("--slots", type=int, default=16, help="request-server slots")
    ap.add_argument("--no-update", action="store_true",
                    help="skip the pattern-change re-ordering of the benchmark mesh")
    ap.add_argument("--no-graph", action="store_true", help="skip the recorded-graph latency")
    ap.add_argument("--no-fill", action="store_true", help="skip the fill-vs-patch-size sweep")
    ap.add_argument("--no-block", action="store_true",
                    help="skip the 2048x2048 torus in 3x3 blocks (12.6M DOF)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter calibration)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two counter runs into profiles/traffic.json and exit")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from(*args.traffic_from, args.copy_probe_mib or 256)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the ordering of one mesh is not sharded across "
              "GPUs in this library (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    A, batch_meshes, serve_reqs = make_inputs(args)
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
    g = run_plain(args, A)
    # the latency-sensitive single-mesh runs first, before the batch, the
    # server and their streams
    modes = None if args.no_fill else run_modes(args, A)
    fill = None if args.no_fill else run_fill(args)
    graph = None if args.no_graph else run_graph(args)
    batch = None if batch_meshes is None else run_batch(args, batch_meshes)
    serving = None if serve_reqs is None else run_serve(args, serve_reqs)
    update = None if args.no_update else run_update(args, A)
    block = None if args.no_block else run_block(args)
    cpu = None if args.no_cpu else run_cpu(A, batch_meshes)
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
                   "depth": g["D"], "nnzL": g["nnzL"], "md_lds_bytes": g["tuning"][0],
                   "md_blocks_per_cu": g["tuning"][1]},
        "roofline": {"bound": "hbm", "kernel": g["dom"], "achieved": round(g["achieved"], 3),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(g["achieved"] / HBM_PEAK_GBS, 6),
                     "traffic": traffic_for(g["dom"]),
                     "bytes_per_launch": round(g["dom_bytes"]),
                     "avg_launch_ms": round(g["dom_avg_ms"], 5),
                     "launches_per_step": g["dom_launches"]},
        # the whole path at the algorithmic bytes per vertex, against the peak
        "path_roofline": {"bytes_per_vertex": round(g["path_bpv"], 2),
                          "boundary_fraction": round(g["beta"], 4),
                          "achieved": round(g["n"] / (g["ms"] * 1e-3) * g["path_bpv"] / 1e9, 3),
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(g["n"] / (g["ms"] * 1e-3) * g["path_bpv"] / 1e9
                                        / HBM_PEAK_GBS, 6)},
        "stage_ms": {k: round(v, 4) for k, v in g["stage_ms"].items()},
        "kernels": g["kernels"],
        "batch": batch,
        "serving": serving,
        "update": update,
        "graph": graph,
        "fill_vs_patch_size": fill,
        "modes": modes,
        "block": block,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
