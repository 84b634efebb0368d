"""GPU: rows wider than the kernels' register windows, against the oracle.

Several stages load a fixed number of a row's entries together and take a
loop for the rest: ingest dedups and ranks rows of up to 16 input entries in
registers, the row scans hold a vertex's first 8 neighbours, the arc
recount a patch's first 16 quotient arcs, and the bisection a node's first
8 local arcs.  These cases put rows exactly at and just past those widths:

- rows of exactly 16 and 17 input entries (the mesh row shuffled, with
  repeated entries), which must give the oracle's result for the clean
  pattern;
- a torus whose every vertex is joined to the 24 others of its 5x5 block,
  with small patches, so every vertex row and most quotient rows are wider
  than the windows.
"""

import numpy as np
import pytest

from paper_2602_00898_amd import meshgen as mg
from tests.gpu_util import compare, cpu_order, gpu_order, mesh, say

pytestmark = pytest.mark.gpu


def padded_rows(A, seed, widths):
    """Each row shuffled and padded with repeats of its own entries to the
    width widths[i] (a row already that wide is only shuffled)."""
    rng = np.random.default_rng(seed)
    rp = A.rowptr.astype(np.int64)
    rows = []
    for i in range(A.n):
        row = A.colind[rp[i]:rp[i + 1]]
        extra = max(0, int(widths[i]) - len(row))
        rows.append(rng.permutation(np.concatenate([row, rng.choice(row, extra)])))
    rp2 = np.zeros(A.n + 1, dtype=np.int64)
    np.cumsum([len(x) for x in rows], out=rp2[1:])
    return mg.CSR(A.n, rp2.astype(np.int32), np.concatenate(rows).astype(np.int32))


def block_stencil_torus(H, W, r):
    """Torus pattern: (i, j) joined to every (i + di, j + dj), |di|, |dj| <= r."""
    idx = np.arange(H * W, dtype=np.int64).reshape(H, W)
    us, vs = [], []
    for di in range(-r, r + 1):
        for dj in range(-r, r + 1):
            if (di, dj) <= (0, 0):
                continue  # each pair once
            us.append(idx.ravel())
            vs.append(np.roll(np.roll(idx, -di, axis=0), -dj, axis=1).ravel())
    return mg.edges_to_csr(H * W, np.concatenate(us), np.concatenate(vs))


@pytest.mark.parametrize("seed", [31, 32])
def test_ingest_rows_of_16_and_17_entries(seed):
    A = mesh(24, 24, True, seed)
    # rows cycle through the widths 16, 17, 7 (as given), 15, 18
    widths = np.array([16, 17, 0, 15, 18])[np.arange(A.n) % 5]
    B = padded_rows(A, seed, widths)
    lens = np.diff(B.rowptr.astype(np.int64))
    assert (lens == 16).any() and (lens == 17).any()
    say(f"[wide] padded rows seed={seed} n={B.n} nnz={B.nnz}")
    compare(gpu_order(B, patch_size=32, seed=seed), cpu_order(A, patch_size=32, seed=seed),
            f"rows of 16/17 entries, seed {seed}")


@pytest.mark.parametrize("H,W,S", [(36, 36, 8), (48, 40, 24)])
def test_every_row_wider_than_the_windows(H, W, S):
    A = block_stencil_torus(H, W, 2)
    assert int(np.diff(A.rowptr.astype(np.int64)).min()) == 25  # 24 neighbours + diagonal
    say(f"[wide] 5x5-block torus {H}x{W} S={S} n={A.n} nnz={A.nnz}")
    compare(gpu_order(A, patch_size=S, seed=5), cpu_order(A, patch_size=S, seed=5),
            f"5x5-block torus {H}x{W} S={S}")
    # the same pattern shuffled and with repeats (ingest's loop path)
    B = padded_rows(A, 7, np.full(A.n, 40))
    compare(gpu_order(B, patch_size=S, seed=5), cpu_order(A, patch_size=S, seed=5),
            f"5x5-block torus {H}x{W} S={S}, rows of 40 entries")
