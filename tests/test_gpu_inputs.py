"""GPU: input format and validation through the C ABI.

The method takes the sparsity pattern of a symmetric matrix (Sec. 4, inputs
and outputs); the order of the entries in a row and repeated entries carry
no information.  So a pattern whose rows are shuffled and partly repeated
must give exactly the oracle's result for the sorted, duplicate-free
pattern, also for rows of more than 512 input entries (a hub vertex, in
scalar and in 3x3 block form, which the ingest handles a workgroup per
row).  With validation on (the default), an asymmetric pattern is refused
with FP_ERR_NOT_SYMMETRIC.
"""

import numpy as np
import pytest

from paper_2602_00898_amd import meshgen as mg
from tests.gpu_util import compare, cpu_order, gpu_order, mesh, say

pytestmark = pytest.mark.gpu


def scramble(A, seed, dup_frac=0.3):
    """Rows shuffled, a fraction of each row's entries repeated."""
    rng = np.random.default_rng(seed)
    rp = A.rowptr.astype(np.int64)
    rows = []
    for i in range(A.n):
        row = A.colind[rp[i]:rp[i + 1]]
        k = int(np.ceil(dup_frac * len(row)))
        rows.append(rng.permutation(np.concatenate([row, rng.choice(row, k)])) if len(row) else row)
    rp2 = np.zeros(A.n + 1, dtype=np.int64)
    np.cumsum([len(x) for x in rows], out=rp2[1:])
    ci = np.concatenate(rows).astype(np.int32) if rows else np.zeros(0, np.int32)
    return mg.CSR(A.n, rp2.astype(np.int32), ci)


def with_hub(A, deg):
    """A plus one extra vertex joined to vertices 0..deg-1 (both ways)."""
    n = A.n + 1
    hub = A.n
    rp = A.rowptr.astype(np.int64)
    rows = []
    for i in range(A.n):
        row = A.colind[rp[i]:rp[i + 1]]
        rows.append(np.append(row, hub) if i < deg else row)
    rows.append(np.append(np.arange(deg), hub))
    rp2 = np.zeros(n + 1, dtype=np.int64)
    np.cumsum([len(x) for x in rows], out=rp2[1:])
    return mg.CSR(n, rp2.astype(np.int32), np.concatenate(rows).astype(np.int32))


def check_same(A_in, A_ref, label, **kw):
    say(f"[inputs] {label} n={A_in.n} nnz={A_in.nnz}")
    g = gpu_order(A_in, **kw)
    c = cpu_order(A_ref, **kw)
    compare(g, c, label)


@pytest.mark.parametrize("H,W,torus,seed,flip,S", [
    (20, 20, True, 8, 0.0, 30),
    (41, 37, False, 9, 0.05, 64),
    (96, 80, True, 10, 0.05, 256),
])
def test_shuffled_and_repeated_entries(H, W, torus, seed, flip, S):
    A = mesh(H, W, torus, seed, flip)
    check_same(scramble(A, seed), A, f"scrambled {H}x{W}", patch_size=S, seed=seed)


def test_long_rows_scalar_and_block():
    A = with_hub(mesh(30, 30, True, 23), 600)
    # the hub row: 600 neighbours + diagonal, each repeated once -> 1202 entries
    B = scramble(A, 5, dup_frac=1.0)
    assert int(B.rowptr[-1] - B.rowptr[-2]) > 512
    check_same(B, A, "hub 600 scrambled", patch_size=64, seed=23)
    Ab = mg.block_expand(A, 3)  # hub rows: 3 x 601 x 3 entries
    Bb = scramble(mg.CSR(Ab.n, Ab.rowptr.astype(np.int64), Ab.colind), 6, dup_frac=0.5)
    Bb = mg.CSR(Bb.n, Bb.rowptr.astype(np.int64), Bb.colind)
    say(f"[inputs] block hub n={Bb.n} nnz={Bb.nnz}")
    g = gpu_order(Bb, patch_size=64, seed=23, block_size=3, rowptr64=True)
    c = cpu_order(Ab, patch_size=64, seed=23, block_size=3)
    compare(g, c, "hub 600 block 3x3 scrambled")


def _raises_not_symmetric(A):
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(A.rowptr.astype(np.int32)).to(dev)
    ci = torch.from_numpy(A.colind.astype(np.int32)).to(dev)
    with pytest.raises(fpm.FpError) as e:
        fpm.order(rp, ci, A.n, patch_size=16)
    assert e.value.code == 2  # FP_ERR_NOT_SYMMETRIC
    torch.cuda.synchronize()


def test_asymmetric_pattern_refused():
    say("[inputs] asymmetric 2-vertex pattern")
    _raises_not_symmetric(mg.CSR(2, np.array([0, 1, 1], np.int32), np.array([1], np.int32)))
    A = mesh(16, 16, True, 24)
    keep = np.ones(A.nnz, bool)
    r = 37
    row = np.arange(A.rowptr[r], A.rowptr[r + 1])
    keep[row[A.colind[row] != r][0]] = False  # drop one off-diagonal entry
    ci = A.colind[keep]
    counts = np.array([keep[A.rowptr[i]:A.rowptr[i + 1]].sum() for i in range(A.n)], np.int64)
    rp = np.zeros(A.n + 1, np.int64)
    np.cumsum(counts, out=rp[1:])
    say("[inputs] torus with one entry dropped")
    _raises_not_symmetric(mg.CSR(A.n, rp.astype(np.int32), ci))
    # the same handle path still orders a valid pattern afterwards
    check_same(A, A, "valid after refusal", patch_size=16, seed=24)
