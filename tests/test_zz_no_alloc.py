"""GPU: fp_order_static (the library's static device scratch, for callers
that cannot allocate) against fp_order (a caller workspace) through the C
ABI, bit-exact, on two calls in a row, the second on a smaller matrix."""

import pytest

from tests.gpu_util import compare, gpu_order, mesh, say

pytestmark = pytest.mark.gpu


def _static_order(A, *, patch_size, seed):
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(A.rowptr).to(dev)
    ci = torch.from_numpy(A.colind).to(dev)
    out = fpm.order_static(rp, ci, A.n, patch_size=patch_size, seed=seed)
    torch.cuda.synchronize()
    r = {k: v.cpu().numpy() for k, v in out.items()}
    nn = int(r["n_nodes"][0])
    r["node_begin"] = r["node_begin"][:nn]
    r["node_size"] = r["node_size"][:nn]
    r["gmap"] = r["gmap"][: A.n]
    r["nnzL"] = int(r["nnzL"][0])
    assert int(r["status"][0]) == 0
    return r


def test_static_scratch_matches_workspace_call():
    cases = [(mesh(160, 144, True, 31, 0.05), 256, 31),  # larger first
             (mesh(40, 36, False, 32, 0.05), 48, 32)]     # then a smaller one
    for A, S, seed in cases:
        say(f"[static] n={A.n} S={S} seed={seed}")
        got = _static_order(A, patch_size=S, seed=seed)
        ref = gpu_order(A, patch_size=S, seed=seed)
        compare(got, ref, f"static n={A.n}")


def test_static_scratch_rejects_oversize():
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    A = mesh(1024, 1024, True, 2)
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(A.rowptr).to(dev)
    ci = torch.from_numpy(A.colind).to(dev)
    with pytest.raises(fpm.FpError) as e:
        fpm.order_static(rp, ci, A.n, patch_size=512, seed=2)
    assert e.value.code == 4  # FP_ERR_SIZE: the workspace would exceed the static scratch
