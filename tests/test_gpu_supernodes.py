"""GPU: supernodal symbolic analysis (fp_supernodes) through the C ABI,
element by element against the oracle's fpo_supernodes.

The GPU call runs on the GPU ordering's parent and colcount (device arrays,
no host round trip); the oracle runs on the oracle ordering's, so the test
covers the ordering and the supernode pass together.  Sizes: small meshes,
the 1024x1024 torus with S = 512, and degenerate inputs.  The 3x3 block
workload is checked in test_gpu_block.py.
"""

import numpy as np
import pytest

import oracle
from tests.gpu_util import mesh, say

pytestmark = pytest.mark.gpu

KEYS = ("Lp", "super_ptr", "super_of", "super_parent", "Lx_ptr")


def gpu_super(parent, colcount):
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    dev = torch.device("cuda:0")
    p = parent if torch.is_tensor(parent) else torch.from_numpy(np.asarray(parent, np.int32)).to(dev)
    c = colcount if torch.is_tensor(colcount) else torch.from_numpy(
        np.asarray(colcount, np.int32)).to(dev)
    out = fpm.supernodes(p, c)
    torch.cuda.synchronize()
    ns = int(out["n_super"].item())
    n = int(p.numel())
    return dict(Lp=out["Lp"].cpu().numpy(), super_ptr=out["super_ptr"][:ns + 1].cpu().numpy(),
                super_of=out["super_of"][:n].cpu().numpy(),
                super_parent=out["super_parent"][:ns].cpu().numpy(),
                Lx_ptr=out["Lx_ptr"][:ns + 1].cpu().numpy(), n_super=ns)


def compare_super(g, c, label):
    assert g["n_super"] == c["n_super"], f"{label}: n_super {g['n_super']} vs {c['n_super']}"
    for k in KEYS:
        a, b = np.asarray(g[k]), np.asarray(c[k])
        assert a.shape == b.shape and np.array_equal(a, b), f"{label}: {k} differs"


def ordered_and_checked(A, S, seed, label):
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(A.rowptr).to(dev)
    ci = torch.from_numpy(A.colind).to(dev)
    out = fpm.order(rp, ci, A.n, patch_size=S, seed=seed)
    g = gpu_super(out["parent"], out["colcount"])
    ref = oracle.order(A.rowptr, A.colind, A.n, patch_size=S, seed=seed)
    c = oracle.supernodes(ref["parent"], ref["colcount"])
    compare_super(g, c, label)
    assert g["Lp"][-1] == ref["nnzL"]
    say(f"[super] {label}: n={A.n} supernodes={g['n_super']}")


@pytest.mark.parametrize("H,W,torus,seed,flip,S", [
    (16, 16, True, 4, 0.0, 16), (40, 40, True, 6, 0.05, 50), (96, 80, True, 7, 0.05, 128),
])
def test_small_meshes(H, W, torus, seed, flip, S):
    ordered_and_checked(mesh(H, W, torus, seed, flip), S, seed, f"{H}x{W}")


def test_torus_1024_S512():
    ordered_and_checked(mesh(1024, 1024, True, 2), 512, 2, "1024x1024 S=512")


def test_degenerate_and_invalid():
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    for parent, cc in (([-1], [1]), ([1, -1], [2, 1]), ([-1, -1, -1], [1, 1, 1]),
                       ([2, 2, -1], [2, 2, 1])):
        compare_super(gpu_super(parent, cc), oracle.supernodes(parent, cc), f"parent {parent}")
    say("[super] invalid parent array")
    dev = torch.device("cuda:0")
    with pytest.raises(fpm.FpError):
        fpm.supernodes(torch.tensor([0, -1], dtype=torch.int32, device=dev),
                       torch.tensor([1, 1], dtype=torch.int32, device=dev))
