"""Pins of the oracle's approximate-minimum-degree local order (F3; Sec. 4.3
Step 4 names AMD; Amestoy, Davis and Duff 1996).

- Where the bound is exact (every variable next to at most one element
  besides the new one: trees, paths, cycles, stars, forests) the order must
  be the exact minimum-degree order, ties to the lowest index.
- On general small graphs the traced bounds are re-derived step by step by
  another route: the elements of the quotient graph are the connected
  components of the eliminated vertices (George and Liu), L_e the live
  vertices next to component e, and A_i the live neighbours of i that share
  no element with i.  Every bound must be at least the exact degree in the
  elimination graph (dense elimination), equal to it where the new element
  is the only one next to i besides at most one other, and the pivot must be
  the least (bound, index).
- The whole ordering with AMD local orders keeps the symbolic outputs exact
  (dense elimination) and a single patch reduces to AMD on the graph.
"""

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import oracle
from tests.test_oracle_pins import mesh_graph, sym_graph


def _edges_tree(rng, n):
    return [(i, int(rng.integers(0, i))) for i in range(1, n)]


@pytest.mark.parametrize("seed", range(6))
def test_amd_equals_md_where_the_bound_is_exact(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 60))
    graphs = [
        _edges_tree(rng, n),                                   # random tree
        [(i, i + 1) for i in range(n - 1)],                    # path
        [(i, (i + 1) % n) for i in range(n)],                  # cycle
        [(0, i) for i in range(1, n)],                         # star
        _edges_tree(rng, n // 2) + [(n // 2 + i, n // 2 + i + 1) for i in range(n - n // 2 - 1)],
    ]
    for edges in graphs:
        perm = rng.permutation(n)  # relabel so ties are not trivial
        rp, ci = sym_graph(n, [(int(perm[a]), int(perm[b])) for a, b in edges])
        assert np.array_equal(oracle.amd(rp, ci), oracle.md(rp, ci))


def _neighbors(rp, ci, v):
    return set(ci[rp[v]:rp[v + 1]].tolist())


def _elements(rp, ci, n, eliminated):
    """Components of the eliminated vertices: list of vertex sets."""
    X = sorted(eliminated)
    if not X:
        return []
    idx = {v: i for i, v in enumerate(X)}
    r, c = [], []
    for v in X:
        for u in _neighbors(rp, ci, v):
            if u in idx:
                r.append(idx[v])
                c.append(idx[u])
    G = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(len(X), len(X)))
    k, lab = connected_components(G, directed=False)
    return [{X[i] for i in range(len(X)) if lab[i] == j} for j in range(k)]


def _exact_degrees(rp, ci, n, order_prefix):
    M = np.zeros((n, n), bool)
    for v in range(n):
        for u in _neighbors(rp, ci, v):
            M[v, u] = True
    alive = np.ones(n, bool)
    for p in order_prefix:
        nb = np.flatnonzero(M[p] & alive)
        nb = nb[nb != p]
        M[np.ix_(nb, nb)] = True
        alive[p] = False
    np.fill_diagonal(M, False)
    return {i: int(np.sum(M[i] & alive)) for i in range(n) if alive[i]}


# densities up to 0.5 so that some variables touch overlapping elements,
# where the bound from the previous degree is the smaller one (seeds 0, 39)
@pytest.mark.parametrize("seed", list(range(8)) + [39])
def test_traced_bound_rederived_from_components(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(8, 28))
    p_edge = float(rng.uniform(0.08, 0.5))
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p_edge]
    rp, ci = sym_graph(n, edges)
    order, T = oracle.amd(rp, ci, trace=True)
    assert np.array_equal(np.sort(order), np.arange(n))
    assert np.array_equal(T[0], [len(_neighbors(rp, ci, v) - {v}) for v in range(n)])
    for k in range(n):
        alive = [i for i in range(n) if i not in set(order[:k].tolist())]
        assert all(T[k][i] >= 0 for i in alive) and all(T[k][i] == -1 for i in order[:k])
        # the pivot: least (bound, index)
        assert order[k] == min(alive, key=lambda i: (T[k][i], i))
        exact = _exact_degrees(rp, ci, n, order[:k].tolist())
        for i in alive:
            assert T[k][i] >= exact[i]
        if k == 0:
            continue
        q = int(order[k - 1])
        elems = _elements(rp, ci, n, order[:k].tolist())
        live = set(alive)
        Lof = [set().union(*(_neighbors(rp, ci, v) for v in e)) & live for e in elems]
        new = next(j for j, e in enumerate(elems) if q in e)
        Lq = Lof[new]
        r = len(alive)
        for i in alive:
            if i not in Lq:
                assert T[k][i] == T[k - 1][i]
                continue
            Ei = [j for j, L in enumerate(Lof) if i in L]
            Ai = {v for v in _neighbors(rp, ci, i) & live
                  if v != i and not any(v in Lof[j] for j in Ei)}
            ext = sum(len(Lof[j] - Lq) for j in Ei if j != new)
            want = min(r - 1, T[k - 1][i] + len(Lq) - 1, len(Ai) + len(Lq) - 1 + ext)
            assert T[k][i] == want, (k, i)
            if len(Ei) <= 2:  # the new element and at most one other
                assert T[k][i] == exact[i]


def test_amd_local_orders_in_the_pipeline():
    A, (rp, ci) = mesh_graph(24, 20, True, 7, 0.05)
    for sched in (0, 1):
        r = oracle.order(A.rowptr, A.colind, A.n, patch_size=16, seed=7, local_amd=True,
                         schedule=sched)
        assert np.array_equal(np.sort(r["perm"]), np.arange(A.n))
        bp, bc, bn = oracle.brute_symbolic(rp, ci, r["perm"])
        assert np.array_equal(r["parent"], bp) and r["nnzL"] == bn
    one = oracle.order(A.rowptr, A.colind, A.n, patch_size=10 ** 6, seed=1, local_amd=True)
    assert one["P"] == 1 and np.array_equal(one["perm"], oracle.amd(rp, ci))


def test_amd_fill_close_to_exact_minimum_degree():
    for H, W, seed in [(40, 40, 1), (64, 48, 2)]:
        A, (rp, ci) = mesh_graph(H, W, True, seed, 0.05)
        fa = oracle.order(A.rowptr, A.colind, A.n, patch_size=10 ** 6, local_amd=True)["nnzL"]
        fm = oracle.order(A.rowptr, A.colind, A.n, patch_size=10 ** 6)["nnzL"]
        assert 0.8 * fm <= fa <= 1.25 * fm
