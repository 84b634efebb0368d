"""GPU parity at the batch and serving workloads' own inputs.

- batch: all 256 seeded meshes (5% edge flips, S from the autotune table)
  ordered in one fp_order_batch call; every mesh's outputs must equal the
  oracle's element for element;
- serving: the first 20 requests of the seeded Poisson stream plus its
  largest request (about 2e6 vertices), submitted together so that they
  overlap on the device; every served result must equal the oracle's.

The oracle runs in a thread pool (its C calls release the interpreter lock
and keep no global state).
"""

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_2602_00898_amd import workloads as wl
from tests.gpu_util import compare, cpu_order, say

pytestmark = pytest.mark.gpu

THREADS = 16


def _batch_dict(out, n):
    r = {k: v.cpu().numpy() for k, v in out.items()}
    nn = int(r["n_nodes"][0])
    r["node_begin"] = r["node_begin"][:nn]
    r["node_size"] = r["node_size"][:nn]
    r["gmap"] = r["gmap"][:n]
    r["nnzL"] = int(r["nnzL"][0])
    return r


def test_batch_workload_256_meshes_match_oracle():
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    specs = wl.batch_specs()
    with ThreadPoolExecutor(THREADS) as ex:
        meshes = list(ex.map(wl.batch_mesh, specs))
    say(f"[batch] {len(meshes)} meshes, {sum(A.n for A in meshes)} vertices generated")
    cfg = [(wl.batch_patch_size(A.n), wl.batch_order_seed(i)) for i, A in enumerate(meshes)]
    dev = torch.device("cuda:0")
    dm = [dict(rowptr=torch.from_numpy(A.rowptr).to(dev), colind=torch.from_numpy(A.colind).to(dev),
               n=A.n, patch_size=S, seed=s) for A, (S, s) in zip(meshes, cfg)]
    outs = fpm.order_batch(dm)
    torch.cuda.synchronize()
    say("[batch] GPU done; oracle")
    with ThreadPoolExecutor(THREADS) as ex:
        refs = list(ex.map(lambda a: cpu_order(a[0], patch_size=a[1][0], seed=a[1][1]),
                           zip(meshes, cfg)))
    for i, (A, out, ref) in enumerate(zip(meshes, outs, refs)):
        compare(_batch_dict(out, A.n), ref, f"batch mesh {i} n={A.n} S={cfg[i][0]}")
    say("[batch] all 256 equal")


def test_serving_workload_requests_match_oracle():
    from paper_2602_00898_amd import fastperm as fpm
    stream = wl.serving_stream(2000)
    largest = max(range(len(stream)), key=lambda i: stream[i][1].n)
    pick = list(range(20)) + ([largest] if largest >= 20 else [])
    specs = [stream[i][1] for i in pick]
    with ThreadPoolExecutor(THREADS) as ex:
        meshes = list(ex.map(wl.serving_mesh, specs))
    say(f"[serve] {len(meshes)} requests, largest n={max(A.n for A in meshes)}")
    srv = fpm.Server(hbm_budget=64 << 30, max_slots=16)
    try:
        tickets = [srv.submit(A.rowptr, A.colind, A.n, patch_size=wl.SERVE_PATCH,
                              seed=wl.SERVE_ORDER_SEED) for A in meshes]
        got = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    say("[serve] served; oracle")
    with ThreadPoolExecutor(THREADS) as ex:
        refs = list(ex.map(lambda A: cpu_order(A, patch_size=wl.SERVE_PATCH,
                                               seed=wl.SERVE_ORDER_SEED), meshes))
    for A, g, c in zip(meshes, got, refs):
        for k in ("perm", "iperm", "parent", "colcount"):
            assert np.array_equal(g[k], c[k]), f"request n={A.n}: {k} differs"
        assert g["nnzL"] == c["nnzL"], f"request n={A.n}: nnzL"
    say("[serve] all requests equal")
