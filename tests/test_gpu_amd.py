"""GPU: approximate-minimum-degree local orders (FP_FLAG_AMD) against the
oracle's AMD mode, element for element: meshes of several sizes and patch
targets, both schedules, with refined separators and a limited depth, 3x3
blocks, a single node of 40,000 vertices (the whole graph as one patch, so
the element arena is compacted many times), a mixed batch and the
1024x1024 torus at S = 512.
"""

import pytest

from paper_2602_00898_amd import meshgen as mg
from tests.gpu_util import compare, cpu_order, gpu_order, mesh, say

pytestmark = pytest.mark.gpu

CASES = [(20, 20, True, 71, 0.05, 8), (41, 37, False, 72, 0.05, 30),
         (96, 80, True, 73, 0.05, 128), (160, 150, False, 74, 0.05, 512)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}S{c[5]}")
def test_amd_local_orders(case):
    H, W, t, s, f, S = case
    A = mesh(H, W, t, s, f)
    for kw in (dict(schedule=0), dict(schedule=1), dict(refine=True, nd_level=3)):
        say(f"[amd] {H}x{W} S={S} {kw}")
        kw = dict(patch_size=S, seed=s, amd=True, **kw)
        compare(gpu_order(A, **kw), cpu_order(A, **kw), f"amd {H}x{W} {kw}")


def test_amd_single_large_node_and_blocks():
    A = mesh(200, 200, True, 75, 0.05)
    say("[amd] one node of 40000 vertices")
    kw = dict(patch_size=10 ** 6, seed=1, amd=True)
    compare(gpu_order(A, **kw), cpu_order(A, **kw), "amd single node")
    B = mg.block_expand(mesh(40, 36, False, 76, 0.05), 3)
    kw = dict(patch_size=32, seed=2, amd=True, block_size=3)
    say("[amd] 3x3 blocks")
    compare(gpu_order(B, **kw), cpu_order(B, **kw), "amd blocks")


def test_amd_batch_and_full_size():
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    from tests.test_gpu_batch import _to_dict
    dev = torch.device("cuda:0")
    specs = [((33, 33, True, 77, 0.05), dict(patch_size=20, seed=1, amd=True)),
             ((50, 40, False, 78, 0.05), dict(patch_size=32, seed=2)),
             ((64, 48, True, 79, 0.05), dict(patch_size=16, seed=3, amd=True, refine=True))]
    ms, cases = [], []
    for geo, kw in specs:
        A = mesh(*geo)
        cases.append((A, kw))
        ms.append(dict(rowptr=torch.from_numpy(A.rowptr).to(dev),
                       colind=torch.from_numpy(A.colind).to(dev), n=A.n, **kw))
    say("[amd] batch of 3")
    for (A, kw), out in zip(cases, fpm.order_batch(ms)):
        compare(_to_dict(out, A), cpu_order(A, **kw), f"amd batch n={A.n}")
    A = mesh(1024, 1024, True, 2)
    say("[amd] 1024x1024 torus S=512")
    kw = dict(patch_size=512, seed=2, amd=True)
    compare(gpu_order(A, **kw), cpu_order(A, **kw), "amd 1024x1024")
