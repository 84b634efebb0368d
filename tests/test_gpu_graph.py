"""GPU: recorded orderings (fp_graph_create / fp_graph_launch).

The whole pipeline of Alg. 1 runs on the device without host work between
its stages, so it can be recorded once into a HIP graph and replayed.  Each
replay must give exactly the oracle's result for the inputs' contents at
that replay (a re-seeded mesh of the same size and entry count is copied in
between replays), with eager work of the same handle and of torch between
the replays, for one matrix and for a batch.
"""

import pytest

from paper_2602_00898_amd import meshgen as mg
from tests.gpu_util import compare, cpu_order, say
from tests.test_gpu_batch import MIX, _to_dict

pytestmark = pytest.mark.gpu


def _dev(A):
    import torch
    dev = torch.device("cuda:0")
    return torch.from_numpy(A.rowptr).to(dev), torch.from_numpy(A.colind).to(dev)


def _eager_between(h, k):
    """Work of the same handle and of torch between two replays."""
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    B = mg.grid_mesh(24 + k, 20, True, 90 + k, 0.05)
    rp, ci = _dev(B)
    out = fpm.order(rp, ci, B.n, patch_size=32, seed=k, handle=h)
    x = torch.arange(1 << 20, device="cuda:0", dtype=torch.float32)
    y = (x * 2).sum()
    torch.cuda.synchronize()
    g = {kk: v.cpu().numpy() for kk, v in out.items()}
    assert int(g["status"][0]) == 0 and float(y) > 0


def test_single_matrix_replays():
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    H, W, S = 48, 40, 64
    seeds = [41, 41, 42, 43, 43]
    A = mg.grid_mesh(H, W, True, seeds[0], 0.05)
    rp, ci = _dev(A)
    h = fpm.Handle()
    g = fpm.Graph([dict(rowptr=rp, colind=ci, n=A.n, patch_size=S, seed=5)], handle=h)
    for r, sd in enumerate(seeds):
        B = mg.grid_mesh(H, W, True, sd, 0.05)
        assert B.n == A.n and B.nnz == A.nnz
        rp.copy_(torch.from_numpy(B.rowptr))
        ci.copy_(torch.from_numpy(B.colind))
        say(f"[graph] single replay {r} mesh seed {sd}")
        outs = g.launch(check=True)
        compare(_to_dict(outs[0], B), cpu_order(B, patch_size=S, seed=5), f"replay {r}")
        _eager_between(h, r)


def test_batch_replays():
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    mix = MIX[:6]
    cases = [(mg.grid_mesh(H, W, t, s, f), S, s) for H, W, t, s, f, S in mix]
    dev = [_dev(A) for A, _, _ in cases]
    h = fpm.Handle()
    g = fpm.Graph([dict(rowptr=rp, colind=ci, n=A.n, patch_size=S, seed=s)
                   for (A, S, s), (rp, ci) in zip(cases, dev)], handle=h)
    for r in range(4):
        # mesh 2 re-seeded from the second replay on (same n and nnz)
        cur = list(cases)
        if r >= 1:
            H, W, t, s, f, S = mix[2]
            B = mg.grid_mesh(H, W, t, s + 100 * r, f)
            assert B.nnz == cases[2][0].nnz
            dev[2][0].copy_(torch.from_numpy(B.rowptr))
            dev[2][1].copy_(torch.from_numpy(B.colind))
            cur[2] = (B, S, s)
        say(f"[graph] batch replay {r}")
        outs = g.launch(check=True)
        for (A, S, s), out in zip(cur, outs):
            compare(_to_dict(out, A), cpu_order(A, patch_size=S, seed=s), f"batch replay {r}")
        _eager_between(h, r)


def test_timing_flag_refused():
    from paper_2602_00898_amd import fastperm as fpm
    A = mg.grid_mesh(16, 16, True, 3, 0.0)
    rp, ci = _dev(A)
    with pytest.raises(fpm.FpError) as e:
        fpm.Graph([dict(rowptr=rp, colind=ci, n=A.n, patch_size=16,
                        flags=fpm.FLAG_TIMING | fpm.FLAG_VALIDATE)])
    assert e.value.code == 1  # FP_ERR_ARG
