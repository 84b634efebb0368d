"""GPU: batched and served orderings through the C ABI.

A matrix ordered inside a batch (every launch covering all matrices), or by
the server next to other requests, must give exactly the result it gets
alone, which is the oracle's.
"""

import numpy as np
import pytest

from paper_2602_00898_amd import meshgen as mg
from tests.gpu_util import compare, cpu_order, gpu_order, mesh, say

pytestmark = pytest.mark.gpu

# (H, W, torus, seed, flip, S): mixed sizes, shapes and patch targets
MIX = [(20, 20, True, 3, 0.05, 40), (9, 30, False, 4, 0.0, 16), (33, 33, True, 5, 0.05, 64),
       (5, 5, False, 6, 0.0, 3), (64, 48, True, 7, 0.05, 128), (3, 3, True, 8, 0.0, 2),
       (100, 90, False, 9, 0.05, 256), (41, 17, True, 10, 0.0, 50)]


def _to_dict(out, A, block_size=1):
    r = {k: v.cpu().numpy() for k, v in out.items()}
    nn = int(r["n_nodes"][0])
    r["node_begin"] = r["node_begin"][:nn]
    r["node_size"] = r["node_size"][:nn]
    r["gmap"] = r["gmap"][: A.n // block_size]
    r["nnzL"] = int(r["nnzL"][0])
    return r


def _device_meshes(cases):
    import torch
    dev = torch.device("cuda:0")
    return [dict(rowptr=torch.from_numpy(A.rowptr).to(dev), colind=torch.from_numpy(A.colind).to(dev),
                 n=A.n, patch_size=S, seed=s) for A, S, s in cases]


@pytest.mark.parametrize("pick", ["all", "reversed", "three"])
def test_batch_matches_oracle_and_single(pick):
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    mix = {"all": MIX, "reversed": MIX[::-1], "three": MIX[2:5]}[pick]
    cases = [(mesh(H, W, t, s, f), S, s) for H, W, t, s, f, S in mix]
    say(f"[batch] {len(cases)} meshes ({pick})")
    outs = fpm.order_batch(_device_meshes(cases))
    torch.cuda.synchronize()
    for (A, S, s), out in zip(cases, outs):
        g = _to_dict(out, A)
        compare(g, cpu_order(A, patch_size=S, seed=s), f"batch n={A.n}")
        compare(g, gpu_order(A, patch_size=S, seed=s), f"batch vs single n={A.n}")


def test_batch_blocks_user_groups_and_options():
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    dev = torch.device("cuda:0")
    B = mg.block_expand(mesh(16, 16, True, 11), 3)
    P = mesh(30, 30, False, 12)
    g = (np.arange(P.n) // 37).astype(np.int32)
    Q = mesh(24, 20, True, 13, 0.05)
    meshes = [
        dict(rowptr=torch.from_numpy(B.rowptr).to(dev), colind=torch.from_numpy(B.colind).to(dev),
             n=B.n, patch_size=40, seed=11, block_size=3),
        dict(rowptr=torch.from_numpy(P.rowptr).to(dev), colind=torch.from_numpy(P.colind).to(dev),
             n=P.n, patch_size=64, user_gmap=torch.from_numpy(g).to(dev)),
        dict(rowptr=torch.from_numpy(Q.rowptr).to(dev), colind=torch.from_numpy(Q.colind).to(dev),
             n=Q.n, patch_size=30, seed=13, schedule=1, lloyd_iters=2),
    ]
    say("[batch] block / user groups / post order")
    outs = fpm.order_batch(meshes)
    torch.cuda.synchronize()
    compare(_to_dict(outs[0], B, 3), cpu_order(B, patch_size=40, seed=11, block_size=3), "block3")
    compare(_to_dict(outs[1], P), cpu_order(P, patch_size=64, user_gmap=g), "user groups")
    compare(_to_dict(outs[2], Q), cpu_order(Q, patch_size=30, seed=13, schedule=1, lloyd_iters=2),
            "post order, lloyd 2")


def test_batch_with_deep_and_shallow_trees():
    """One batch whose meshes take the levels past their expected depth in
    different ways: a mesh with 150 isolated vertices next to ordinary ones."""
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    A = mesh(16, 16, True, 27)
    iso = 150
    rp = np.concatenate([A.rowptr[:-1], A.nnz + np.arange(iso + 1)]).astype(np.int32)
    ci = np.concatenate([A.colind, A.n + np.arange(iso)]).astype(np.int32)
    deep = mg.CSR(A.n + iso, rp, ci)
    cases = [(mesh(20, 20, True, 3, 0.05), 40, 3), (deep, 300, 4), (mesh(33, 33, True, 5, 0.05), 64, 5)]
    say("[batch] deep and shallow trees")
    outs = fpm.order_batch(_device_meshes(cases))
    torch.cuda.synchronize()
    for (M, S, s), out in zip(cases, outs):
        compare(_to_dict(out, M), cpu_order(M, patch_size=S, seed=s), f"batch n={M.n}")


def test_batch_concatenated_arrays():
    """fp_order_batch_concat over one concatenated CSR (local indices per
    mesh) gives each mesh its own fp_order result, in the concatenated
    outputs."""
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    cases = [(mesh(H, W, t, s, f), S, s) for H, W, t, s, f, S in MIX]
    rp = np.concatenate([A.rowptr.astype(np.int64) for A, _, _ in cases])
    ci = np.concatenate([A.colind for A, _, _ in cases]).astype(np.int32)
    vo = np.concatenate([[0], np.cumsum([A.n for A, _, _ in cases])])
    no = np.concatenate([[0], np.cumsum([A.nnz for A, _, _ in cases])])
    dev = torch.device("cuda:0")
    say(f"[batch] concatenated: {len(cases)} meshes, {vo[-1]} vertices")
    out = fpm.order_batch_concat(torch.from_numpy(rp).to(dev), torch.from_numpy(ci).to(dev), vo, no,
                                 [dict(patch_size=S, seed=s) for _, S, s in cases])
    r = {k: v.cpu().numpy() for k, v in out.items() if torch.is_tensor(v)}
    for i, (A, S, s) in enumerate(cases):
        c = cpu_order(A, patch_size=S, seed=s)
        sl = slice(vo[i], vo[i + 1])
        for k in ("perm", "iperm", "parent", "colcount"):
            assert np.array_equal(r[k][sl], c[k]), f"concat mesh {i}: {k}"
        assert int(r["nnzL"][i]) == c["nnzL"] and int(r["status"][i]) == 0
        nn = len(c["node_begin"])
        no_i = int(out["node_off"][i])
        assert np.array_equal(r["node_begin"][no_i:no_i + nn], c["node_begin"])
        assert np.array_equal(r["node_size"][no_i:no_i + nn], c["node_size"])


def test_server_same_alone_and_in_mix():
    from paper_2602_00898_amd import fastperm as fpm
    target = mesh(70, 60, True, 21, 0.05)
    S = 100
    srv = fpm.Server(hbm_budget=1 << 30, max_slots=4)
    try:
        say("[server] target alone")
        t = srv.submit(target.rowptr, target.colind, target.n, patch_size=S, seed=21)
        alone = srv.wait(t)
        say("[server] target among 11 other requests")
        mix = [(mesh(H, W, tt, s, f), SS, s) for H, W, tt, s, f, SS in MIX]
        tickets = [srv.submit(A.rowptr, A.colind, A.n, patch_size=SS, seed=s) for A, SS, s in mix[:4]]
        tt_target = srv.submit(target.rowptr, target.colind, target.n, patch_size=S, seed=21)
        tickets += [srv.submit(A.rowptr, A.colind, A.n, patch_size=SS, seed=s) for A, SS, s in mix[4:]]
        inmix = srv.wait(tt_target)
        for (A, SS, s), tk in zip(mix, tickets):
            r = srv.wait(tk)
            c = cpu_order(A, patch_size=SS, seed=s)
            for k in ("perm", "iperm", "parent", "colcount"):
                assert np.array_equal(r[k], c[k]), f"server n={A.n}: {k}"
            assert r["nnzL"] == c["nnzL"]
            assert r["latency_s"] > 0
    finally:
        srv.close()
    c = cpu_order(target, patch_size=S, seed=21)
    for k in ("perm", "iperm", "parent", "colcount"):
        assert np.array_equal(alone[k], c[k]), f"alone: {k}"
        assert np.array_equal(inmix[k], alone[k]), f"in the mix: {k}"
    assert alone["nnzL"] == inmix["nnzL"] == c["nnzL"]


def test_server_refuses_oversize_request():
    from paper_2602_00898_amd import fastperm as fpm
    A = mesh(64, 64, True, 22)
    srv = fpm.Server(hbm_budget=1 << 16, max_slots=1)
    try:
        with pytest.raises(fpm.FpError) as e:
            srv.submit(A.rowptr, A.colind, A.n, patch_size=64)
        assert e.value.code == 7  # FP_ERR_BUSY
    finally:
        srv.close()


def test_server_small_requests_pass_a_waiting_large_one():
    """Under a budget that holds one large request but not two, the second
    large request waits for memory while the small ones behind it are
    admitted; every result still equals the oracle's."""
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    big = [mesh(300, 280, True, 31, 0.05), mesh(290, 300, False, 32, 0.05)]
    small = [mesh(30 + 3 * i, 28, True, 40 + i, 0.05) for i in range(6)]
    h = fpm.Handle()
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(big[0].rowptr).to(dev)
    ci = torch.from_numpy(big[0].colind).to(dev)
    ws, _ = fpm.query(h, big[0].n, rp, ci, fpm.options(128))
    foot = ws + 40 * big[0].n + 8 * big[0].nnz  # about the server's own estimate
    srv = fpm.Server(hbm_budget=int(1.6 * foot), max_slots=4)
    try:
        say("[server] 2 large + 6 small requests under a tight budget")
        reqs = [(A, 128, 31 + i) for i, A in enumerate(big)] + [(A, 32, 50 + i) for i, A in enumerate(small)]
        tickets = [srv.submit(A.rowptr, A.colind, A.n, patch_size=S, seed=s) for A, S, s in reqs]
        for (A, S, s), tk in zip(reqs, tickets):
            r = srv.wait(tk)
            c = cpu_order(A, patch_size=S, seed=s)
            for k in ("perm", "iperm", "parent", "colcount"):
                assert np.array_equal(r[k], c[k]), f"server n={A.n}: {k}"
            assert r["nnzL"] == c["nnzL"]
    finally:
        srv.close()


def test_batch_reuses_outputs():
    """A second batch call on the outputs of the first (outs=) writes the
    same results into them."""
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    cases = [(mesh(H, W, t, s, f), S, s) for H, W, t, s, f, S in MIX[:4]]
    say("[batch] outputs reused")
    h = fpm.Handle()
    dm = _device_meshes(cases)
    outs = fpm.order_batch(dm, handle=h)
    for o in outs:
        o["perm"].fill_(-1)
        o["parent"].fill_(-7)
    again = fpm.order_batch(dm, handle=h, outs=outs)
    torch.cuda.synchronize()
    assert all(a["perm"] is b["perm"] for a, b in zip(outs, again))
    for (A, S, s), out in zip(cases, again):
        compare(_to_dict(out, A), cpu_order(A, patch_size=S, seed=s), f"reused n={A.n}")
