"""The seeded input generators: the row-by-row builder used for large
serving requests gives exactly the pattern of the edge-list builder, and the
workload recipes are deterministic per seed."""

import numpy as np
import pytest

from paper_2602_00898_amd import meshgen as mg


@pytest.mark.parametrize("H,W,torus,seed", [(3, 3, True, 1), (4, 7, False, 2), (17, 16, True, 3),
                                            (33, 30, False, 4), (64, 64, True, 5),
                                            (101, 97, False, 6)])
def test_direct_builder_equals_edge_list_builder(H, W, torus, seed):
    a = mg.grid_mesh(H, W, torus, seed)
    b = mg.grid_mesh_direct(H, W, torus, seed, index64=True)
    assert a.n == b.n
    assert np.array_equal(a.rowptr.astype(np.int64), b.rowptr)
    assert np.array_equal(a.colind, b.colind)


def test_workload_recipes_are_deterministic():
    a, b = mg.batch_specs(3), mg.batch_specs(3)
    assert [(m.side, m.torus, m.seed) for m in a] == [(m.side, m.torus, m.seed) for m in b]
    assert len(a) == 256 and all(45 <= m.side <= 447 for m in a)
    s1, s2 = mg.serving_stream(5, 50), mg.serving_stream(5, 50)
    assert [(t, m.side, m.seed) for t, m in s1] == [(t, m.side, m.seed) for t, m in s2]
    assert all(100 <= m.side <= 1414 for _, m in s1)
    assert all(t2 > t1 for (t1, _), (t2, _) in zip(s1, s1[1:]))


def test_swap_quad_diagonals_is_a_local_symmetric_change():
    import scipy.sparse as sp
    A = mg.grid_mesh(12, 10, True, 3)
    B = mg.swap_quad_diagonals(A, 10, [(2, 3), (7, 9)])
    M = sp.csr_matrix((np.ones(B.nnz), B.colind, B.rowptr), shape=(B.n, B.n))
    assert (M != M.T).nnz == 0 and B.nnz == A.nnz
    MA = sp.csr_matrix((np.ones(A.nnz), A.colind, A.rowptr), shape=(A.n, A.n))
    assert (M != MA).nnz == 8  # two edges out, two in, both directions
    C = mg.swap_quad_diagonals(B, 10, [(2, 3), (7, 9)])
    assert np.array_equal(C.rowptr, A.rowptr) and np.array_equal(C.colind, A.colind)
