"""GPU: fixed recursion depth and refined separators against the oracle.

nd_level (Sec. 4.2, Step 3) stops the nested dissection after that many
levels, each leaf keeping the remaining vertices of all its patches;
FP_FLAG_REFINE takes the smallest separator inside the superset (Sec. 5,
separator refinement), computed on the device by a parallel maximum
matching whose canonical cover does not depend on the matching found.
Every output must equal the oracle's element for element: single matrices
(scalar and 3x3 blocks, both schedules, depths from 0 to the full depth),
a batch mixing the modes, and the 1024x1024 torus at S = 512 refined.
"""

import numpy as np
import pytest

from paper_2602_00898_amd import meshgen as mg
from tests.gpu_util import compare, cpu_order, gpu_order, mesh, say

pytestmark = pytest.mark.gpu

CASES = [  # H, W, torus, seed, flip, S
    (20, 20, True, 51, 0.05, 8), (41, 37, False, 52, 0.05, 30), (64, 64, True, 53, 0.05, 64),
    (128, 96, False, 54, 0.05, 128), (200, 200, True, 55, 0.05, 256)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}S{c[5]}")
def test_refined_separators(case):
    H, W, t, s, f, S = case
    A = mesh(H, W, t, s, f)
    for sched in (0, 1):
        say(f"[refine] {H}x{W} S={S} sched={sched}")
        kw = dict(patch_size=S, seed=s, schedule=sched, refine=True)
        compare(gpu_order(A, **kw), cpu_order(A, **kw), f"refine {H}x{W} sched {sched}")


@pytest.mark.parametrize("refine", [False, True])
@pytest.mark.parametrize("case", CASES[1:4], ids=lambda c: f"{c[0]}x{c[1]}S{c[5]}")
def test_limited_depth(case, refine):
    H, W, t, s, f, S = case
    A = mesh(H, W, t, s, f)
    full = cpu_order(A, patch_size=S, seed=s)
    for L in sorted({0 if A.n <= 4096 else 1, 1, 3, max(full["D"] - 2, 0), full["D"] - 1,
                     full["D"] + 1}):
        say(f"[nd_level] {H}x{W} S={S} nd_level={L} refine={refine}")
        kw = dict(patch_size=S, seed=s, nd_level=L, refine=refine)
        c = cpu_order(A, **kw)
        assert c["D"] == min(L, full["D"])
        compare(gpu_order(A, **kw), c, f"nd_level {L} {H}x{W}")


def test_blocks_post_order_limited_refined():
    A = mesh(48, 40, True, 56, 0.05)
    B = mg.block_expand(A, 3)
    kw = dict(patch_size=24, seed=56, block_size=3, schedule=1, nd_level=3, refine=True)
    say("[refine] block 3x3 48x40 nd_level=3 post order")
    compare(gpu_order(B, **kw), cpu_order(B, **kw), "block refine")


def test_batch_mixing_modes():
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    from tests.test_gpu_batch import _to_dict
    dev = torch.device("cuda:0")
    specs = [((33, 33, True, 61, 0.05), dict(patch_size=20, seed=1, refine=True)),
             ((50, 40, False, 62, 0.05), dict(patch_size=32, seed=2, nd_level=2)),
             ((64, 48, True, 63, 0.05), dict(patch_size=16, seed=3)),
             ((90, 90, True, 64, 0.05), dict(patch_size=64, seed=4, nd_level=4, refine=True)),
             ((9, 9, False, 65, 0.0), dict(patch_size=4, seed=5, refine=True, schedule=1))]
    meshes, ms = [], []
    for geo, kw in specs:
        A = mesh(*geo)
        meshes.append((A, kw))
        ms.append(dict(rowptr=torch.from_numpy(A.rowptr).to(dev),
                       colind=torch.from_numpy(A.colind).to(dev), n=A.n, **kw))
    say("[refine] batch of 5 mixed modes")
    outs = fpm.order_batch(ms)
    for (A, kw), out in zip(meshes, outs):
        compare(_to_dict(out, A), cpu_order(A, **kw), f"batch n={A.n} {kw}")


def test_refined_full_size_torus():
    A = mesh(1024, 1024, True, 2)
    say("[refine] 1024x1024 torus S=512 refined")
    g = gpu_order(A, patch_size=512, seed=2, refine=True)
    c = cpu_order(A, patch_size=512, seed=2, refine=True)
    compare(g, c, "1024x1024 refined")
    base = cpu_order(A, patch_size=512, seed=2)
    say(f"[refine] nnz(L) one-sided {base['nnzL']} refined {c['nnzL']}")
    root = lambda r: int(r["node_size"][0])  # noqa: E731
    assert root(c) <= root(base)
    assert np.array_equal(np.sort(g["perm"]), np.arange(A.n))
