"""CPU pins of the oracle's supernodal symbolic analysis (fundamental
supernodes, Liu, Ng and Peyton 1993), which the solver's symbolic phase
builds from the elimination tree (Sec. 1).

The oracle derives supernodes from parent and column counts alone.  The
pins rebuild every column structure of L by dense boolean elimination and
apply the definition set by set: columns j and j+1 share a supernode iff j
is the only child of j+1 and struct(L_j) = {j} + struct(L_{j+1}).  Hand
cases (a path, a clique, a star, a forest) fix the boundary values.
"""

import numpy as np
import pytest

import oracle
from paper_2602_00898_amd import meshgen as mg


def dense_structures(grp, gci, perm):
    """Boolean column structures of L for A(perm, perm): list of sorted row
    index arrays (diagonal included)."""
    n = len(grp) - 1
    ip = np.empty(n, np.int64)
    ip[perm] = np.arange(n)
    M = np.zeros((n, n), bool)
    for v in range(n):
        for e in range(grp[v], grp[v + 1]):
            i, j = ip[v], ip[gci[e]]
            M[i, j] = M[j, i] = True
    cols = []
    for j in range(n):
        below = np.flatnonzero(M[j + 1:, j]) + j + 1
        cols.append(np.concatenate([[j], below]))
        # eliminating j joins its later neighbours into a clique
        if len(below):
            M[np.ix_(below, below)] = True
    return cols


def by_definition(cols):
    n = len(cols)
    parent = np.array([c[1] if len(c) > 1 else -1 for c in cols])
    nchild = np.bincount(parent[parent >= 0], minlength=n) if n else np.zeros(0, int)
    starts = [0]
    for j in range(n - 1):
        same = (parent[j] == j + 1 and nchild[j + 1] == 1
                and set(cols[j][1:].tolist()) == set(cols[j + 1].tolist()))
        if not same:
            starts.append(j + 1)
    sptr = np.array(starts + [n])
    sof = np.repeat(np.arange(len(starts)), np.diff(sptr))
    spar = np.array([-1 if len(cols[sptr[s + 1] - 1]) == 1 else sof[cols[sptr[s + 1] - 1][1]]
                     for s in range(len(starts))])
    rows = np.array([len(cols[sptr[s]]) for s in range(len(starts))], np.int64)
    lx = np.concatenate([[0], np.cumsum(rows * np.diff(sptr))])
    lp = np.concatenate([[0], np.cumsum([len(c) for c in cols])])
    return dict(parent=parent, colcount=np.array([len(c) for c in cols]), super_ptr=sptr,
                super_of=sof, super_parent=spar, Lx_ptr=lx, Lp=lp)


def check(grp, gci, perm):
    cols = dense_structures(grp, gci, perm)
    ref = by_definition(cols)
    got = oracle.supernodes(ref["parent"], ref["colcount"])
    for k in ("Lp", "super_of", "super_ptr", "super_parent", "Lx_ptr"):
        assert np.array_equal(got[k], ref[k]), k
    assert got["n_super"] == len(ref["super_ptr"]) - 1
    return got


def graph_of(edges, n):
    adj = [set() for _ in range(n)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    grp = np.zeros(n + 1, np.int64)
    np.cumsum([len(a) for a in adj], out=grp[1:])
    gci = np.array([x for a in adj for x in sorted(a)], np.int32)
    return grp, gci


def test_hand_cases():
    n = 6
    # path in natural order: a chain, column counts 2,...,2,1; only the last
    # two columns merge
    g = check(*graph_of([(i, i + 1) for i in range(n - 1)], n), np.arange(n))
    assert g["n_super"] == n - 1
    assert list(g["super_ptr"]) == [0, 1, 2, 3, 4, 6]
    # clique: one supernode holding every column, a dense triangle stored
    # as an n x n block
    g = check(*graph_of([(i, j) for i in range(n) for j in range(i + 1, n)], n), np.arange(n))
    assert g["n_super"] == 1 and list(g["Lx_ptr"]) == [0, n * n]
    # star with the centre last: each leaf its own supernode, the centre too
    g = check(*graph_of([(i, n - 1) for i in range(n - 1)], n), np.arange(n))
    assert g["n_super"] == n and list(g["super_parent"]) == [n - 1] * (n - 1) + [-1]
    # a forest of isolated vertices: every column a root supernode
    g = check(np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.arange(n))
    assert g["n_super"] == n and all(g["super_parent"] == -1)


@pytest.mark.parametrize("seed", range(6))
def test_random_graph_random_order(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 60))
    m = int(rng.integers(0, 3 * n))
    edges = {(int(a), int(b)) for a, b in rng.integers(0, n, (m, 2)) if a != b}
    grp, gci = graph_of(edges, n)
    check(grp, gci, rng.permutation(n).astype(np.int32))


@pytest.mark.parametrize("H,W,torus,seed,S", [(12, 12, True, 1, 16), (20, 16, False, 2, 32),
                                              (24, 24, True, 3, 64)])
def test_mesh_orderings(H, W, torus, seed, S):
    A = mg.grid_mesh(H, W, torus, seed, 0.05)
    r = oracle.order(A.rowptr, A.colind, A.n, patch_size=S, seed=seed)
    grp, gci = oracle.graph(A.rowptr, A.colind, A.n)
    g = check(grp, gci, r["perm"])
    assert g["Lp"][-1] == r["nnzL"]


def test_invariants_on_a_larger_ordering():
    A = mg.grid_mesh(128, 128, True, 4, 0.05)
    r = oracle.order(A.rowptr, A.colind, A.n, patch_size=256, seed=4)
    g = oracle.supernodes(r["parent"], r["colcount"])
    sp, spar, sof = g["super_ptr"], g["super_parent"], g["super_of"]
    assert sp[0] == 0 and sp[-1] == A.n and np.all(np.diff(sp) >= 1)
    assert np.all((spar == -1) | (spar > np.arange(len(spar))))
    assert g["Lp"][-1] == r["nnzL"]
    # inside a supernode the etree is a chain and the counts drop by one
    inner = np.flatnonzero(np.diff(sof) == 0)
    assert np.all(r["parent"][inner] == inner + 1)
    assert np.all(r["colcount"][inner] == r["colcount"][inner + 1] + 1)
    # roots of the supernodal tree = roots of the etree
    assert np.sum(spar == -1) == np.sum(r["parent"] == -1)
