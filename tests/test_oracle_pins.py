"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test re-derives a result by a different route than the oracle's code:
library shortest paths (scipy), dense elimination, declarative re-statement
of a definition from the final outputs, closed forms and hand cases.
"""

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, shortest_path

import oracle
from paper_2602_00898_amd import meshgen as mg


# ---------------------------------------------------------------- helpers

def sym_graph(n, edges):
    """CSR (int64 rowptr, int32 colind) of an undirected simple graph."""
    if len(edges) == 0:
        return np.zeros(n + 1, dtype=np.int64), np.zeros(0, dtype=np.int32)
    e = np.asarray(edges, dtype=np.int64)
    r = np.concatenate([e[:, 0], e[:, 1]])
    c = np.concatenate([e[:, 1], e[:, 0]])
    keep = r != c
    key = np.unique(r[keep] * n + c[keep])
    r, c = key // n, key % n
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=rp[1:])
    return rp, c.astype(np.int32)


def random_graph(rng, n, p, extra_components=0):
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    return sym_graph(n, edges)


def mesh_graph(H, W, torus, seed, flip=0.0):
    A = mg.grid_mesh(H, W, torus, seed, flip)
    return A, oracle.graph(A.rowptr, A.colind, A.n)


def to_scipy(rp, ci):
    n = len(rp) - 1
    return sp.csr_matrix((np.ones(len(ci)), ci, rp), shape=(n, n))


def hop_dist(rp, ci, sources=None):
    d = shortest_path(to_scipy(rp, ci), unweighted=True, directed=False, indices=sources)
    return d


MESHES = [(8, 8, False, 11), (9, 7, True, 12), (16, 16, True, 13), (12, 20, False, 14),
          (24, 24, True, 15)]


# ---------------------------------------------------------------- O0, hash

def test_mix64_published_values():
    # SplitMix64 seeded with 0: the first outputs of the published generator
    assert oracle.mix64(0, 0) == 0xE220A8397B1DCDAF
    assert oracle.mix64(0, 1) == 0x6E789E6AA1B965F4
    assert oracle.mix64(0, 2) == 0x06C45D188009454F


def test_graph_strips_diagonal_dedups_and_sorts():
    A = mg.grid_mesh(10, 10, True, 3)
    grp, gci = oracle.graph(A.rowptr, A.colind, A.n)
    # scrambled copy: reversed rows, every entry twice
    rp, ci = A.rowptr.astype(np.int64), A.colind
    rows = [np.concatenate([ci[rp[i]:rp[i + 1]][::-1], ci[rp[i]:rp[i + 1]]]) for i in range(A.n)]
    rp2 = np.zeros(A.n + 1, dtype=np.int64)
    np.cumsum([len(r) for r in rows], out=rp2[1:])
    g2 = oracle.graph(rp2, np.concatenate(rows), A.n)
    assert np.array_equal(grp, g2[0]) and np.array_equal(gci, g2[1])
    for i in range(A.n):
        row = gci[grp[i]:grp[i + 1]]
        assert i not in row and np.all(np.diff(row) > 0)
    assert len(gci) == 2 * 3 * A.n


def test_graph_block_compression_matches_vertex_graph():
    A = mg.grid_mesh(7, 9, True, 4)
    B = mg.block_expand(A, 3)
    g1 = oracle.graph(A.rowptr, A.colind, A.n)
    g3 = oracle.graph(B.rowptr, B.colind, B.n, block_size=3)
    assert np.array_equal(g1[0], g3[0]) and np.array_equal(g1[1], g3[1])


# ---------------------------------------------------------------- O1 patches

@pytest.mark.parametrize("seed", range(6))
def test_grow_is_nearest_seed_lowest_id(seed):
    rng = np.random.default_rng(seed)
    if seed % 2:
        _, (rp, ci) = mesh_graph(11, 13, bool(seed % 3), seed, 0.05)
    else:
        rp, ci = random_graph(rng, 60, 0.05)
    n = len(rp) - 1
    seeds = rng.choice(n, size=7, replace=False).astype(np.int32)
    lab = oracle.grow(rp, ci, seeds)
    d = hop_dist(rp, ci, seeds)  # (k, n)
    for v in range(n):
        dv = d[:, v]
        if np.all(np.isinf(dv)):
            assert lab[v] == -1
        else:
            best = min(range(len(seeds)), key=lambda k: (dv[k], k))
            assert lab[v] == best


def test_seed_selection_without_lloyd():
    A, (rp, ci) = mesh_graph(20, 20, True, 5)
    S, sigma = 37, 99
    gmap, seeds = oracle.patches(rp, ci, S, lloyd_iters=0, seed=sigma)
    P0 = -(-A.n // S)
    h = mg._mix64(sigma, np.arange(A.n))
    for b in range(P0):
        ids = np.arange(b * S, min(A.n, (b + 1) * S))
        assert seeds[b] == ids[np.argmin(h[ids])]
    assert len(seeds) == P0
    assert np.array_equal(gmap, oracle.grow(rp, ci, seeds))


@pytest.mark.parametrize("mesh", MESHES)
@pytest.mark.parametrize("S", [5, 16, 40])
def test_patches_invariants_and_lloyd_rule(mesh, S):
    A, (rp, ci) = mesh_graph(*mesh)
    n = A.n
    g0, s0 = oracle.patches(rp, ci, S, lloyd_iters=0, seed=7)
    g1, s1 = oracle.patches(rp, ci, S, lloyd_iters=1, seed=7)
    P = len(s1)
    assert P == len(s0) >= -(-n // S)
    assert g1.min() == 0 and g1.max() == P - 1 and len(np.unique(g1)) == P
    G = to_scipy(rp, ci)
    for k in range(P):
        idx = np.flatnonzero(g1 == k)
        nc, _ = connected_components(G[idx][:, idx], directed=False)
        assert nc == 1
    # Lloyd: new seed of patch k = farthest member (intra-patch hops) from
    # the members having a neighbour in another patch; ties to the lowest id
    for k in range(P):
        idx = np.flatnonzero(g0 == k)
        sub = G[idx][:, idx]
        bnd = [i for i, v in enumerate(idx) if np.any(g0[ci[rp[v]:rp[v + 1]]] != k)]
        if not bnd:
            assert s1[k] == s0[k]
            continue
        dist = shortest_path(sub, unweighted=True, directed=False, indices=bnd).min(axis=0)
        best = max(range(len(idx)), key=lambda i: (dist[i], -idx[i]))
        assert s1[k] == idx[best]
    assert np.array_equal(g1, oracle.grow(rp, ci, s1))


def test_orphan_components_become_patches():
    # two meshes side by side plus isolated vertices, one seed block: the
    # components without the seed become patches in order of lowest id
    A, (rp1, ci1) = mesh_graph(10, 10, False, 1)
    n1 = A.n
    rp = np.concatenate([rp1, rp1[-1] + rp1[1:], np.full(3, 2 * rp1[-1])]).astype(np.int64)
    ci = np.concatenate([ci1, ci1 + n1]).astype(np.int32)
    n = 2 * n1 + 3
    assert len(rp) == n + 1
    _, s0 = oracle.patches(rp, ci, 1000, lloyd_iters=0, seed=3)
    gmap, seeds = oracle.patches(rp, ci, 1000, lloyd_iters=1, seed=3)
    nc, comp = connected_components(to_scipy(rp, ci), directed=False)
    assert nc == 5 and len(seeds) == 5
    first = comp[s0[0]]
    others = sorted((c for c in range(nc) if c != first), key=lambda c: np.flatnonzero(comp == c).min())
    expect = np.empty(n, dtype=np.int32)
    expect[comp == first] = 0
    for k, c in enumerate(others):
        expect[comp == c] = k + 1
    assert np.array_equal(gmap, expect)


# ---------------------------------------------------------------- O4 bisect

def brute_bisect(w, rp, ci):
    m = len(w)
    G = to_scipy(rp, ci)
    dist = shortest_path(G, unweighted=True, directed=False)
    deg = np.diff(rp)
    nc, comp = connected_components(G, directed=False)
    order_comp = sorted(range(nc), key=lambda c: np.flatnonzero(comp == c).min())
    Q = []
    for c in order_comp:
        mem = np.flatnonzero(comp == c)
        r = mem.min()
        ecc = lambda x: int(dist[x, mem].max())  # noqa: E731
        er = ecc(r)
        for _ in range(8):
            last = [x for x in mem if dist[r, x] == er]
            cnd = min(last, key=lambda x: (deg[x], x))
            if ecc(cnd) > er:
                r, er = cnd, ecc(cnd)
            else:
                break
        Q += sorted(mem, key=lambda x: (dist[r, x], x))
    W = int(np.sum(w))
    if W == 0:
        ks = (m + 1) // 2
    else:
        ks = next((k for k in range(1, m + 1) if 2 * sum(w[Q[i]] for i in range(k)) >= W), m)
    h = int(np.ceil(np.log2(m)))
    cap = 2 ** (h - 1)
    k = min(max(ks, max(1, m - cap)), min(m - 1, cap))
    left = np.zeros(m, dtype=bool)
    left[Q[:k]] = True
    return left


def random_tree(rng, m):
    # random labels so the lowest id sits anywhere in the tree
    lab = rng.permutation(m)
    edges = [(int(lab[i]), int(lab[int(rng.integers(max(0, i - 3), i))])) for i in range(1, m)]
    return sym_graph(m, edges)


@pytest.mark.parametrize("seed", range(60))
def test_bisect_matches_distance_based_rederivation(seed):
    rng = np.random.default_rng(100 + seed)
    m = int(rng.integers(2, 40))
    if seed % 4 == 1:
        rp, ci = random_tree(rng, m)
    elif seed % 3 == 0:
        _, (rp, ci) = mesh_graph(int(rng.integers(2, 7)), int(rng.integers(2, 7)), False, seed)
        m = len(rp) - 1
    else:
        rp, ci = random_graph(rng, m, float(rng.uniform(0.02, 0.3)))
    w = rng.integers(0, 20, size=m).astype(np.int64)
    if seed % 5 == 0:
        w[:] = 0
    left = oracle.bisect(w, rp, ci)
    assert np.array_equal(left, brute_bisect(w, rp, ci))
    h = int(np.ceil(np.log2(m)))
    assert 1 <= left.sum() <= 2 ** (h - 1) and 1 <= (~left).sum() <= 2 ** (h - 1)


# ---------------------------------------------------------------- O2-O6 septree

def subtree(t, nn):
    out, st = [], [t]
    while st:
        x = st.pop()
        if x < nn:
            out.append(x)
            st += [2 * x + 1, 2 * x + 2]
    return set(out)


def check_septree(rp, ci, gmap, P, node_of, pnode, D, one_sided=True):
    n = len(rp) - 1
    nn = 2 ** (D + 1) - 1
    assert np.all((node_of >= 0) & (node_of < nn))
    # every patch ends at one node whose subtree-capacity holds
    depth = lambda t: int(np.floor(np.log2(t + 1)))  # noqa: E731
    for p in range(P):
        assert 0 <= pnode[p] < nn
    for t in range(nn):
        assert np.sum(pnode == t) <= 1 or D == 0
    # unmarked vertices sit at their patch's node, separators at ancestors
    for v in range(n):
        t, leaf = node_of[v], pnode[gmap[v]]
        a = leaf
        while a != t and a > 0:
            a = (a - 1) // 2
        assert a == t, "separator node is not an ancestor of the patch node"
    sub = {t: subtree(t, nn) for t in range(nn)}
    for t in range(nn):
        if 2 * t + 2 >= nn:
            continue
        L, R = sub[2 * t + 1], sub[2 * t + 2]
        inL = np.isin(node_of, list(L))
        inR = np.isin(node_of, list(R))
        # nested-dissection property: no edge between the two subtrees
        for v in np.flatnonzero(inL):
            assert not np.any(inR[ci[rp[v]:rp[v + 1]]])
        # separator = one side's candidate set, the smaller (ties left)
        U = np.isin(node_of, list(sub[t]))
        if not np.any(U):
            continue
        sideL = np.isin(pnode[gmap], list(L))
        sideR = np.isin(pnode[gmap], list(R))
        cand_L = {v for v in np.flatnonzero(U & sideL)
                  if np.any(U[ci[rp[v]:rp[v + 1]]] & sideR[ci[rp[v]:rp[v + 1]]])}
        cand_R = {v for v in np.flatnonzero(U & sideR)
                  if np.any(U[ci[rp[v]:rp[v + 1]]] & sideL[ci[rp[v]:rp[v + 1]]])}
        M = set(np.flatnonzero(node_of == t))
        pt = set(np.flatnonzero(np.isin(pnode, list(sub[t]))))
        if len(pt) >= 2:
            if one_sided:
                assert M == (cand_L if len(cand_L) <= len(cand_R) else cand_R)
            else:
                assert M <= cand_L | cand_R
            # the split of the patches is the bisection of the quotient
            # subgraph as it stood before this level
            pl = sorted(pt)
            loc = {p: i for i, p in enumerate(pl)}
            wv = np.array([np.sum(U & (gmap == p)) for p in pl], dtype=np.int64)
            edges = set()
            for v in np.flatnonzero(U):
                for u in ci[rp[v]:rp[v + 1]]:
                    if U[u] and gmap[u] != gmap[v]:
                        edges.add((loc[gmap[v]], loc[gmap[u]]))
            arp, aci = sym_graph(len(pl), sorted(edges))
            left = oracle.bisect(wv, arp, aci)
            got = np.array([pnode[p] in L for p in pl])
            assert np.array_equal(left, got)
        elif len(pt) == 1:
            # a single patch is not split: the node is its leaf
            assert all(pnode[p] == t for p in pt)
        else:
            assert not M


@pytest.mark.parametrize("mesh", MESHES[:4])
@pytest.mark.parametrize("S", [6, 20])
def test_septree_definition_and_nd_property(mesh, S):
    A, (rp, ci) = mesh_graph(*mesh)
    gmap, seeds = oracle.patches(rp, ci, S, 1, 5)
    P = len(seeds)
    node_of, pnode, D = oracle.septree(rp, ci, gmap, P)
    assert D == int(np.ceil(np.log2(P))) if P > 1 else D == 0
    check_septree(rp, ci, gmap, P, node_of, pnode, D)


def test_septree_disconnected_user_groups():
    A, (rp, ci) = mesh_graph(12, 12, False, 8)
    rng = np.random.default_rng(1)
    gmap = rng.integers(0, 9, size=A.n).astype(np.int32)  # disconnected groups
    node_of, pnode, D = oracle.septree(rp, ci, gmap, 9)
    check_septree(rp, ci, gmap, 9, node_of, pnode, D)


# ---------------------------------------------------------------- O7 MD

def test_md_hand_cases():
    path = sym_graph(5, [(0, 1), (1, 2), (2, 3), (3, 4)])
    assert list(oracle.md(*path)) == [0, 1, 2, 3, 4]
    star = sym_graph(5, [(0, 1), (0, 2), (0, 3), (0, 4)])
    assert list(oracle.md(*star)) == [1, 2, 3, 0, 4]
    clique = sym_graph(6, [(i, j) for i in range(6) for j in range(i + 1, 6)])
    assert list(oracle.md(*clique)) == list(range(6))
    cycle = sym_graph(6, [(i, (i + 1) % 6) for i in range(6)])
    # all degree 2: 0 first; its neighbours 1 and 5 join (degree stays 2)
    assert list(oracle.md(*cycle)) == [0, 1, 2, 3, 4, 5]
    assert len(oracle.md(np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32))) == 0


@pytest.mark.parametrize("seed", range(30))
def test_md_matches_dense_recomputation(seed):
    rng = np.random.default_rng(seed)
    if seed % 3 == 0:
        _, (rp, ci) = mesh_graph(int(rng.integers(3, 12)), int(rng.integers(3, 12)),
                                 bool(seed % 2), seed, 0.05)
    else:
        rp, ci = random_graph(rng, int(rng.integers(1, 70)), float(rng.uniform(0.01, 0.3)))
    assert np.array_equal(oracle.md(rp, ci), oracle.brute_md(rp, ci))


@pytest.mark.parametrize("seed", range(5))
def test_md_forest_has_no_fill(seed):
    rng = np.random.default_rng(seed)
    n = 80
    edges = [(i, int(rng.integers(0, i))) for i in range(1, n) if rng.random() < 0.9]
    rp, ci = sym_graph(n, edges)
    order = oracle.md(rp, ci)
    _, _, nnzL = oracle.brute_symbolic(rp, ci, order)
    assert nnzL == n + len(edges)


# ---------------------------------------------------------------- O9, O10

@pytest.mark.parametrize("seed", range(8))
def test_etree_colcount_match_dense_elimination_random_perm(seed):
    rng = np.random.default_rng(seed)
    if seed % 2:
        _, (rp, ci) = mesh_graph(15, 17, True, seed, 0.05)
    else:
        rp, ci = random_graph(rng, 150, 0.03)
    n = len(rp) - 1
    perm = rng.permutation(n).astype(np.int32)
    par = oracle.etree(rp, ci, perm)
    cc, nnz = oracle.colcount(rp, ci, perm, par)
    bp, bc, bn = oracle.brute_symbolic(rp, ci, perm)
    assert np.array_equal(par, bp) and np.array_equal(cc, bc) and nnz == bn


def test_c1_ordering_matches_dense_elimination():
    """64x64 planar grid, seeded diagonals, S = 64 (the tiny configuration)."""
    A = mg.grid_mesh(64, 64, False, 1)
    r = oracle.order(A.rowptr, A.colind, A.n, patch_size=64, seed=1)
    rp, ci = oracle.graph(A.rowptr, A.colind, A.n)
    assert np.array_equal(np.sort(r["perm"]), np.arange(A.n))
    assert np.array_equal(r["iperm"][r["perm"]], np.arange(A.n))
    bp, bc, bn = oracle.brute_symbolic(rp, ci, r["perm"])
    assert np.array_equal(r["parent"], bp)
    assert np.array_equal(r["colcount"], bc)
    assert r["nnzL"] == bn
    check_septree(rp, ci, r["gmap"], r["P"], r["node_of"], _pnode_from(r, rp, ci), r["D"])


def _pnode_from(r, rp, ci):
    """Final node of each patch, from the separator tree of the same gmap."""
    node_of, pnode, D = oracle.septree(rp, ci, r["gmap"], r["P"])
    assert np.array_equal(node_of, r["node_of"]) and D == r["D"]
    return pnode


def test_symbolic_invariants_on_larger_mesh():
    A, (rp, ci) = mesh_graph(96, 96, True, 9, 0.05)
    r = oracle.order(A.rowptr, A.colind, A.n, patch_size=128, seed=9)
    par, cc = r["parent"], r["colcount"]
    n = A.n
    ok = par >= 0
    assert np.all(par[ok] > np.arange(n)[ok])
    assert np.sum(~ok) == connected_components(to_scipy(rp, ci), directed=False)[0]
    # struct(L_j) minus j is contained in struct(L_parent(j))
    assert np.all(cc[par[ok]] >= cc[ok] - 1)
    # column count at least the below-diagonal entries of A(perm, perm)
    ip = r["iperm"]
    for j in range(0, n, 97):
        v = r["perm"][j]
        below = np.sum(ip[ci[rp[v]:rp[v + 1]]] > j)
        assert cc[j] >= 1 + below


# ---------------------------------------------------------------- O8 schedules

@pytest.mark.parametrize("mesh", MESHES[2:])
def test_level_and_post_order_same_fill(mesh):
    A, (rp, ci) = mesh_graph(*mesh)
    a = oracle.order(A.rowptr, A.colind, A.n, patch_size=24, seed=4, schedule=oracle.SCHED_LEVEL)
    b = oracle.order(A.rowptr, A.colind, A.n, patch_size=24, seed=4, schedule=oracle.SCHED_POST)
    assert a["nnzL"] == b["nnzL"]
    # per original vertex the column count is the same
    assert np.array_equal(a["colcount"][a["iperm"]], b["colcount"][b["iperm"]])
    for r in (a, b):
        nb, ns = r["node_begin"], r["node_size"]
        for t in range(1, r["n_nodes"]):
            par = (t - 1) // 2
            if ns[t] and ns[par]:
                assert nb[t] + ns[t] <= nb[par]
        # perm blocks are the nodes
        for t in range(r["n_nodes"]):
            blk = r["perm"][nb[t]:nb[t] + ns[t]]
            assert np.all(r["node_of"][blk] == t)


def _schedule_sequence(D, sched):
    """Node sequence of a schedule over the heap of depth D, from its
    definition: level order lists depth D first, then D-1, ..., 0, each depth
    by ascending heap index; post order visits the left subtree, the right
    subtree, then the node."""
    if sched == oracle.SCHED_LEVEL:
        return [t for d in range(D, -1, -1) for t in range((1 << d) - 1, (1 << (d + 1)) - 1)]
    seq, nn = [], (1 << (D + 1)) - 1
    stack = [(0, False)]
    while stack:
        t, done = stack.pop()
        if t >= nn:
            continue
        if done:
            seq.append(t)
        else:
            stack += [(t, True), (2 * t + 2, False), (2 * t + 1, False)]
    return seq


@pytest.mark.parametrize("sched", [oracle.SCHED_LEVEL, oracle.SCHED_POST])
@pytest.mark.parametrize("mesh,S", [((16, 16, True, 13), 24), ((12, 20, False, 14), 7),
                                    ((24, 24, True, 15), 40), ((20, 21, False, 16), 3)])
def test_concatenation_sequence_exact(mesh, S, sched):
    """perm is the concatenation of the local orders along the schedule
    (Alg. 3): rebuilt here from node_of, the schedule's definition and the
    minimum-degree order of each node's induced subgraph, it must equal the
    oracle's perm and node ranges element for element."""
    A, (rp, ci) = mesh_graph(*mesh)
    r = oracle.order(A.rowptr, A.colind, A.n, patch_size=S, seed=5, schedule=sched)
    D, nof = r["D"], r["node_of"]
    seq = _schedule_sequence(D, sched)
    assert sorted(seq) == list(range((1 << (D + 1)) - 1))
    begin = np.zeros(len(seq), dtype=np.int64)
    perm = []
    for t in seq:
        begin[t] = len(perm)
        V = np.flatnonzero(nof == t)  # ascending ids = local indices
        if len(V) == 0:
            continue
        loc = -np.ones(A.n, dtype=np.int64)
        loc[V] = np.arange(len(V))
        rows = [[loc[u] for u in ci[rp[v]:rp[v + 1]] if loc[u] >= 0] for v in V]
        lrp = np.zeros(len(V) + 1, dtype=np.int64)
        np.cumsum([len(x) for x in rows], out=lrp[1:])
        lci = np.array([x for row in rows for x in row], dtype=np.int32)
        perm.extend(V[oracle.brute_md(lrp, lci)])
    assert np.array_equal(np.asarray(perm), r["perm"])
    assert np.array_equal(begin, r["node_begin"])
    assert np.array_equal(np.bincount(nof, minlength=len(seq)), r["node_size"])


# ---------------------------------------------------------------- limits, blocks

def test_single_patch_reduces_to_minimum_degree():
    A, (rp, ci) = mesh_graph(9, 11, True, 2)
    r = oracle.order(A.rowptr, A.colind, A.n, patch_size=10 ** 6, seed=1)
    assert r["P"] == 1 and r["D"] == 0
    assert np.array_equal(r["perm"], oracle.md(rp, ci))


def test_patch_size_one_is_classical_nested_dissection():
    A, (rp, ci) = mesh_graph(10, 10, False, 3)
    r = oracle.order(A.rowptr, A.colind, A.n, patch_size=1, seed=1)
    assert r["P"] == A.n
    assert np.array_equal(r["gmap"], np.arange(A.n))  # each vertex its own patch
    pn = _pnode_from(r, rp, ci)
    check_septree(rp, ci, r["gmap"], r["P"], r["node_of"], pn, r["D"])
    bp, bc, bn = oracle.brute_symbolic(rp, ci, r["perm"])
    assert np.array_equal(r["parent"], bp) and r["nnzL"] == bn


@pytest.mark.parametrize("sched", [oracle.SCHED_LEVEL, oracle.SCHED_POST])
def test_block_expansion_equals_dof_symbolic(sched):
    A = mg.grid_mesh(10, 12, True, 6)
    B = mg.block_expand(A, 3)
    rv = oracle.order(A.rowptr, A.colind, A.n, patch_size=16, seed=6, schedule=sched)
    rb = oracle.order(B.rowptr, B.colind, B.n, patch_size=16, seed=6, schedule=sched,
                      block_size=3)
    assert np.array_equal(rb["perm"][0::3], 3 * rv["perm"])
    drp, dci = oracle.graph(B.rowptr, B.colind, B.n)
    bp, bc, bn = oracle.brute_symbolic(drp, dci, rb["perm"])
    assert np.array_equal(rb["parent"], bp)
    assert np.array_equal(rb["colcount"], bc)
    assert rb["nnzL"] == bn == 9 * rv["nnzL"] - 3 * A.n


def test_user_gmap_reproduces_patching():
    A = mg.grid_mesh(30, 30, True, 7)
    r = oracle.order(A.rowptr, A.colind, A.n, patch_size=50, seed=7)
    u = oracle.order(A.rowptr, A.colind, A.n, patch_size=50, seed=7, user_gmap=r["gmap"])
    for k in ("perm", "parent", "colcount"):
        assert np.array_equal(r[k], u[k])


def test_input_order_and_duplicates_do_not_matter():
    A = mg.grid_mesh(20, 20, True, 8)
    rng = np.random.default_rng(0)
    rp = A.rowptr.astype(np.int64)
    rows = []
    for i in range(A.n):
        row = A.colind[rp[i]:rp[i + 1]]
        row = np.concatenate([row, row[:2]])
        rows.append(rng.permutation(row))
    rp2 = np.zeros(A.n + 1, dtype=np.int64)
    np.cumsum([len(x) for x in rows], out=rp2[1:])
    a = oracle.order(A.rowptr, A.colind, A.n, patch_size=30, seed=1)
    b = oracle.order(rp2, np.concatenate(rows), A.n, patch_size=30, seed=1)
    for k in ("perm", "parent", "colcount", "gmap", "node_of"):
        assert np.array_equal(a[k], b[k])


def test_long_rows_order_and_duplicates_do_not_matter():
    """A vertex of degree 600 whose row is shuffled and every entry repeated
    (1202 entries) gives the same ordering as the clean pattern."""
    A = mg.grid_mesh(30, 30, True, 23)
    hub, deg = A.n, 600
    rp = A.rowptr.astype(np.int64)
    rows = [np.append(A.colind[rp[i]:rp[i + 1]], hub) if i < deg else A.colind[rp[i]:rp[i + 1]]
            for i in range(A.n)]
    rows.append(np.append(np.arange(deg), hub))
    rng = np.random.default_rng(3)
    messy = [rng.permutation(np.concatenate([r, r])) for r in rows]

    def csr(rr):
        p = np.zeros(len(rr) + 1, dtype=np.int64)
        np.cumsum([len(x) for x in rr], out=p[1:])
        return p, np.concatenate(rr).astype(np.int32)

    a = oracle.order(*csr(rows), A.n + 1, patch_size=64, seed=23)
    b = oracle.order(*csr(messy), A.n + 1, patch_size=64, seed=23)
    for k in ("perm", "parent", "colcount", "gmap", "node_of"):
        assert np.array_equal(a[k], b[k])


def test_errors():
    A = mg.grid_mesh(5, 5, False, 1)
    bad = A.colind.copy()
    bad[3] = A.n + 5
    with pytest.raises(RuntimeError):
        oracle.order(A.rowptr, bad, A.n)
    with pytest.raises(RuntimeError):
        oracle.order(A.rowptr, A.colind, A.n, patch_size=0)
    with pytest.raises(RuntimeError):  # not symmetric
        rp = np.array([0, 1, 1], dtype=np.int64)
        oracle.order(rp, np.array([1], dtype=np.int32), 2)
    empty = oracle.order(np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32), 0)
    assert empty["nnzL"] == 0 and empty["P"] == 0
    one = oracle.order(np.array([0, 1]), np.array([0], dtype=np.int32), 1)
    assert list(one["perm"]) == [0] and list(one["parent"]) == [-1] and one["nnzL"] == 1
