"""Shared helpers of the GPU parity tests: run the HIP path and the oracle on
the same seeded input and compare element by element."""

import sys

import numpy as np

import oracle
from paper_2602_00898_amd import meshgen as mg

FIELDS = ("gmap", "node_begin", "node_size", "perm", "iperm", "parent", "colcount")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_order(A, *, patch_size, seed=0, schedule=0, block_size=1, lloyd_iters=1, user_gmap=None,
              rowptr64=False, handle=None, nd_level=-1, refine=False, amd=False):
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(A.rowptr.astype(np.int64 if rowptr64 else np.int32)).to(dev)
    ci = torch.from_numpy(A.colind.astype(np.int32)).to(dev)
    ug = None if user_gmap is None else torch.from_numpy(np.asarray(user_gmap, np.int32)).to(dev)
    out = fpm.order(rp, ci, A.n, patch_size=patch_size, seed=seed, schedule=schedule,
                    block_size=block_size, lloyd_iters=lloyd_iters, user_gmap=ug, handle=handle,
                    nd_level=nd_level, refine=refine, amd=amd)
    torch.cuda.synchronize()
    r = {k: v.cpu().numpy() for k, v in out.items()}
    nn = int(r["n_nodes"][0])
    r["node_begin"] = r["node_begin"][:nn]
    r["node_size"] = r["node_size"][:nn]
    r["gmap"] = r["gmap"][: A.n // block_size]
    r["nnzL"] = int(r["nnzL"][0])
    return r


def cpu_order(A, *, patch_size, seed=0, schedule=0, block_size=1, lloyd_iters=1, user_gmap=None,
              nd_level=-1, refine=False, amd=False, **_):
    return oracle.order(A.rowptr, A.colind, A.n, patch_size=patch_size, seed=seed,
                        schedule=schedule, block_size=block_size, lloyd_iters=lloyd_iters,
                        user_gmap=user_gmap, nd_level=nd_level, refine=refine,
                        local_amd=amd)


def compare(g, c, label=""):
    """Bit-exact comparison; reports the first field that differs."""
    for k in FIELDS:
        a, b = np.asarray(g[k]), np.asarray(c[k])
        if a.shape != b.shape or not np.array_equal(a, b):
            bad = np.flatnonzero(a != b) if a.shape == b.shape else []
            i = bad[0] if len(bad) else None
            raise AssertionError(f"{label}: field {k} differs (shape {a.shape} vs {b.shape}; "
                                 f"{len(bad)} mismatches; first at {i}: "
                                 f"{a[i] if i is not None else ''} vs {b[i] if i is not None else ''})")
    assert g["nnzL"] == c["nnzL"], f"{label}: nnzL {g['nnzL']} vs {c['nnzL']}"


def mesh(H, W, torus, seed, flip=0.0):
    return mg.grid_mesh(H, W, torus, seed, flip)
