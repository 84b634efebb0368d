"""GPU: re-ordering after a pattern change with the patches kept
(fp_order_update), through the C ABI.

The result must equal the oracle's ordering of the new pattern with the
earlier call's patches as user groups (Sec. 5 user-provided groups), element
by element.  Local orders of unchanged separator-tree nodes are reused: for
an unchanged pattern every vertex's order is reused, for a local change most
are, and a call whose vertex count differs reuses nothing.
"""

import numpy as np
import pytest

from paper_2602_00898_amd import meshgen as mg
from tests.gpu_util import compare, cpu_order, mesh, say

pytestmark = pytest.mark.gpu


def _dev(A):
    import torch
    dev = torch.device("cuda:0")
    return torch.from_numpy(A.rowptr).to(dev), torch.from_numpy(A.colind).to(dev)


def _dict(out, n):
    r = {k: v.cpu().numpy() for k, v in out.items()}
    nn = int(r["n_nodes"][0])
    r["node_begin"] = r["node_begin"][:nn]
    r["node_size"] = r["node_size"][:nn]
    r["gmap"] = r["gmap"][:n]
    r["nnzL"] = int(r["nnzL"][0])
    return r


@pytest.mark.parametrize("H,W,seed,S,quads", [
    (48, 40, 31, 64, [(3, 4), (3, 6)]),
    (96, 80, 32, 128, [(10, 10), (11, 12), (40, 60)]),
    (160, 144, 33, 256, []),
])
def test_update_matches_oracle_with_kept_patches(H, W, seed, S, quads):
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    A = mesh(H, W, True, seed, 0.05)
    h0, h1 = fpm.Handle(), fpm.Handle()
    rp, ci = _dev(A)
    first = fpm.order(rp, ci, A.n, patch_size=S, seed=seed, handle=h0)
    gmap = first["gmap"][:A.n].clone()
    B = mg.swap_quad_diagonals(A, W, quads) if quads else A
    say(f"[update] {H}x{W} S={S}: {len(quads)} quads changed")
    rp2, ci2 = _dev(B)
    out = fpm.order_update(rp2, ci2, B.n, gmap, h0._ws, patch_size=S, seed=seed, handle=h1)
    torch.cuda.synchronize()
    reused = int(out.pop("reused").item())
    got = _dict(out, B.n)
    ref = cpu_order(B, patch_size=S, user_gmap=gmap.cpu().numpy())
    compare(got, ref, f"update {H}x{W}")
    say(f"[update] reused {reused} of {B.n} vertices")
    if not quads:
        assert reused == B.n
        assert np.array_equal(got["perm"], first["perm"].cpu().numpy())
    else:
        assert 0 < reused < B.n


def test_update_other_size_reuses_nothing():
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    A = mesh(40, 40, True, 34)
    B = mesh(40, 41, True, 35)
    h0, h1 = fpm.Handle(), fpm.Handle()
    rp, ci = _dev(A)
    fpm.order(rp, ci, A.n, patch_size=64, seed=34, handle=h0)
    gB = (np.arange(B.n) // 50).astype(np.int32)
    rp2, ci2 = _dev(B)
    gdev = torch.from_numpy(gB).to(torch.device("cuda:0"))
    out = fpm.order_update(rp2, ci2, B.n, gdev, h0._ws, patch_size=64, handle=h1)
    torch.cuda.synchronize()
    assert int(out.pop("reused").item()) == 0
    compare(_dict(out, B.n), cpu_order(B, patch_size=64, user_gmap=gB), "other size")
