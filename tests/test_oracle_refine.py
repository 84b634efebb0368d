"""Pins of the oracle's fixed recursion depth and refined separators.

nd_level (Sec. 4.2, Step 3): the recursion stops after nd_level levels and
each leaf keeps the remaining vertices of all its patches.  The levels above
the limit are computed exactly as without it, so the limited tree is the
full tree cut at depth nd_level: a pin that relates the two modes without
re-typing either.  nd_level = 0 leaves one node, whose local order is the
minimum-degree order of the whole graph.

Refined separators (Sec. 5, separator refinement; read as the smallest
separator inside the superset, since both sides follow the patches): the
separator of a node must cover every crossing edge, have the size of a
maximum matching of the crossing graph (Konig's theorem; sizes from scipy's
maximum_bipartite_matching, or from subset enumeration on tiny graphs), and
be the canonical cover (s-side candidates that every maximum matching
covers, plus the other-side neighbours of the rest), whose s-side part is
re-derived here vertex by vertex from matching sizes (v is left free by
some maximum matching iff removing v keeps the matching number).
"""

import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import maximum_bipartite_matching

import oracle
from paper_2602_00898_amd import meshgen as mg
from tests.test_oracle_pins import MESHES, check_septree, mesh_graph, subtree, sym_graph


def ancestor_at(t, depth):
    while t > 0 and int(np.floor(np.log2(t + 1))) > depth:
        t = (t - 1) // 2
    return t


# ---------------------------------------------------------------- nd_level

@pytest.mark.parametrize("mesh", MESHES[2:])
@pytest.mark.parametrize("S", [6, 16])
def test_limited_depth_is_the_full_tree_cut(mesh, S):
    A, (rp, ci) = mesh_graph(*mesh)
    gmap, seeds = oracle.patches(rp, ci, S, 1, 3)
    P = len(seeds)
    full, pfull, D = oracle.septree(rp, ci, gmap, P)
    for L in range(0, D + 2):
        node_of, pnode, DL = oracle.septree(rp, ci, gmap, P, nd_level=L)
        assert DL == min(D, L)
        want = np.array([ancestor_at(t, DL) for t in full])
        assert np.array_equal(node_of, want), f"nd_level={L}"
        assert np.array_equal(pnode, [ancestor_at(t, DL) for t in pfull])
        if L >= D:
            assert np.array_equal(node_of, full)


@pytest.mark.parametrize("refine", [False, True])
def test_limited_depth_orderings(refine):
    A, (rp, ci) = mesh_graph(24, 24, True, 15, 0.05)
    base = oracle.order(A.rowptr, A.colind, A.n, patch_size=8, seed=2, refine=refine)
    assert base["D"] >= 5
    for L in (0, 2, base["D"] - 1, base["D"], 30):
        r = oracle.order(A.rowptr, A.colind, A.n, patch_size=8, seed=2, nd_level=L,
                         refine=refine)
        assert r["D"] == min(base["D"], L) and r["n_nodes"] == 2 ** (r["D"] + 1) - 1
        assert np.array_equal(np.sort(r["perm"]), np.arange(A.n))
        bp, bc, bn = oracle.brute_symbolic(rp, ci, r["perm"])
        assert np.array_equal(r["parent"], bp) and np.array_equal(r["colcount"], bc)
        assert r["nnzL"] == bn
        if L >= base["D"]:
            assert np.array_equal(r["perm"], base["perm"])
        # leaves hold every patch below them: sizes add up
        nn = r["n_nodes"]
        assert r["node_size"][:nn].sum() == A.n
    r0 = oracle.order(A.rowptr, A.colind, A.n, patch_size=8, seed=2, nd_level=0)
    assert np.array_equal(r0["perm"], oracle.md(rp, ci))


def test_limited_depth_with_post_order_and_blocks():
    A = mg.grid_mesh(14, 12, False, 4, 0.05)
    B = mg.block_expand(A, 3)
    v = oracle.order(A.rowptr, A.colind, A.n, patch_size=6, seed=1, nd_level=2, schedule=1)
    b = oracle.order(B.rowptr, B.colind, B.n, patch_size=6, seed=1, nd_level=2, schedule=1,
                     block_size=3)
    k = np.arange(A.n)
    for r in range(3):
        assert np.array_equal(b["perm"][3 * k + r], 3 * v["perm"] + r)
    assert b["nnzL"] == 9 * v["nnzL"] - 3 * A.n


# ---------------------------------------------------------------- refinement

def crossing(rp, ci, U, sideS, sideO):
    """Candidates of the s side and the other side and the crossing edges
    between unmarked vertices (U) of the two sides."""
    edges = set()
    for v in np.flatnonzero(U & sideS):
        for u in ci[rp[v]:rp[v + 1]]:
            if U[u] and sideO[u]:
                edges.add((int(v), int(u)))
    cs = sorted({a for a, _ in edges})
    co = sorted({b for _, b in edges})
    return cs, co, sorted(edges)


def matching_number(cs, co, edges, drop=None):
    if not edges:
        return 0
    ri = {v: i for i, v in enumerate(cs)}
    ro = {v: i for i, v in enumerate(co)}
    e = [(ri[a], ro[b]) for a, b in edges if a != drop and b != drop]
    if not e:
        return 0
    r = np.array([x for x, _ in e])
    c = np.array([y for _, y in e])
    B = sp.csr_matrix((np.ones(len(e)), (r, c)), shape=(len(cs), len(co)))
    return int(np.sum(maximum_bipartite_matching(B, perm_type="column") >= 0))


def expected_cover(cs, co, edges):
    """(s-side vertices matched by every maximum matching) plus the other-side
    neighbours of the s-vertices that some maximum matching leaves free."""
    nu = matching_number(cs, co, edges)
    free_some = {v for v in cs if matching_number(cs, co, edges, drop=v) == nu}
    nbr = {b for a, b in edges if a in free_some}
    return (set(cs) - free_some) | nbr, nu


def check_refined(rp, ci, gmap, P, node_of, pnode, D):
    n = len(rp) - 1
    nn = 2 ** (D + 1) - 1
    sub = {t: subtree(t, nn) for t in range(nn)}
    for t in range(nn):
        if 2 * t + 2 >= nn:
            continue
        L, R = sub[2 * t + 1], sub[2 * t + 2]
        U = np.isin(node_of, list(sub[t]))
        pt = set(np.flatnonzero(np.isin(pnode, list(sub[t]))))
        if not np.any(U) or len(pt) < 2:
            continue
        sideL = np.isin(pnode[gmap], list(L))
        sideR = np.isin(pnode[gmap], list(R))
        cl, _, _ = crossing(rp, ci, U, sideL, sideR)
        cr, _, _ = crossing(rp, ci, U, sideR, sideL)
        s_left = len(cl) <= len(cr)
        cs, co, edges = crossing(rp, ci, U, sideL if s_left else sideR, sideR if s_left else sideL)
        M = set(np.flatnonzero(node_of == t).tolist())
        want, nu = expected_cover(cs, co, edges)
        assert len(M) == nu, f"node {t}: separator {len(M)} vs matching number {nu}"
        assert M == want, f"node {t}: not the canonical minimum cover"
        assert len(M) <= min(len(cl), len(cr))
    assert n == len(node_of)


@pytest.mark.parametrize("mesh", MESHES[:4])
@pytest.mark.parametrize("S", [6, 20])
def test_refined_separators_are_canonical_minimum_covers(mesh, S):
    A, (rp, ci) = mesh_graph(*mesh)
    gmap, seeds = oracle.patches(rp, ci, S, 1, 5)
    P = len(seeds)
    node_of, pnode, D = oracle.septree(rp, ci, gmap, P, refine=True)
    check_septree(rp, ci, gmap, P, node_of, pnode, D, one_sided=False)
    check_refined(rp, ci, gmap, P, node_of, pnode, D)


def _two_groups(rng, a, b, p):
    """Groups 0 (vertices 0..a-1) and 1 (a..a+b-1), each a path, with random
    crossing edges of density p."""
    edges = [(i, i + 1) for i in range(a - 1)] + [(a + i, a + i + 1) for i in range(b - 1)]
    cross = [(i, a + j) for i in range(a) for j in range(b) if rng.random() < p]
    rp, ci = sym_graph(a + b, edges + cross)
    gmap = np.array([0] * a + [1] * b, dtype=np.int32)
    return rp, ci, gmap, cross


@pytest.mark.parametrize("seed", range(8))
def test_refined_root_against_brute_force_cover(seed):
    rng = np.random.default_rng(seed)
    a, b = int(rng.integers(3, 8)), int(rng.integers(3, 8))
    rp, ci, gmap, cross = _two_groups(rng, a, b, 0.3)
    node_of, pnode, D = oracle.septree(rp, ci, gmap, 2, refine=True)
    assert D == 1
    M = set(np.flatnonzero(node_of == 0).tolist())
    # every crossing edge covered, and no smaller cover exists (enumeration)
    assert all(u in M or v in M for u, v in cross)
    verts = sorted({x for e in cross for x in e})
    best = next(k for k in range(len(verts) + 1)
                for c in itertools.combinations(verts, k)
                if all(u in c or v in c for u, v in cross))
    assert len(M) == best
    one, _, _ = oracle.septree(rp, ci, gmap, 2)
    assert len(M) <= int(np.sum(one == 0))


def test_refinement_never_enlarges_the_root_separator():
    for H, W, torus, seed in [(32, 32, True, 1), (40, 24, False, 2), (48, 48, True, 3)]:
        A, (rp, ci) = mesh_graph(H, W, torus, seed, 0.05)
        gmap, seeds = oracle.patches(rp, ci, 24, 1, seed)
        one, _, _ = oracle.septree(rp, ci, gmap, len(seeds))
        ref, _, _ = oracle.septree(rp, ci, gmap, len(seeds), refine=True)
        assert np.sum(ref == 0) <= np.sum(one == 0)


def test_refined_ordering_symbolic_exact():
    A, (rp, ci) = mesh_graph(20, 18, False, 6, 0.05)
    for sched in (0, 1):
        r = oracle.order(A.rowptr, A.colind, A.n, patch_size=8, seed=6, refine=True,
                         schedule=sched)
        bp, bc, bn = oracle.brute_symbolic(rp, ci, r["perm"])
        assert np.array_equal(r["parent"], bp) and r["nnzL"] == bn
