"""Seeded synthetic triangle-mesh patterns (input generation only).

This module builds the *inputs* that both the GPU path and the CPU oracle
consume: grid and torus triangle meshes whose quads are split along a seeded
diagonal, optional seeded edge flips, the matrix pattern (vertex adjacency
plus the diagonal) as CSR, the dense b x b block expansion of a pattern, and
the request mixes used for batching and serving.  It holds none of the
ordering method's arithmetic.

Stand-in for the paper's scanned meshes (Sec. 6: Smithsonian, ThreeDScans,
Thingi10K), which are not available: grids and tori have the same vertex
degree distribution (4..8, mean 6) as typical triangle meshes.

Vertex id of grid point (r, c) is r * W + c.  Quad (r, c) has corners
(r, c), (r, c+1), (r+1, c), (r+1, c+1); bit 0 of mix64(seed, quad id) picks
the diagonal (r, c)-(r+1, c+1) when 0 and (r, c+1)-(r+1, c) when 1.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)


def _mix64(seed: int, idx: np.ndarray) -> np.ndarray:
    """SplitMix64 output number idx+1 of a generator seeded with ``seed``.

    Steele, Lea and Flood, "Fast splittable pseudorandom number generators"
    (OOPSLA 2014): state advances by the golden-ratio increment and the
    output is the variant-13 finaliser.
    """
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (idx.astype(np.uint64) + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


@dataclass
class CSR:
    """Symmetric sparsity pattern in CSR form (host numpy arrays)."""

    n: int
    rowptr: np.ndarray  # int32 or int64, n+1
    colind: np.ndarray  # int32, nnz

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


def grid_edges(H: int, W: int, torus: bool, seed: int, flip_frac: float = 0.0):
    """Undirected edge list (u < v not required) of a seeded grid/torus mesh.

    Returns (u, v) int64 arrays.  ``flip_frac`` is the fraction of all edges
    that get flipped: flips act on horizontal grid edges (r, c)-(r, c+1) with
    r and c even, 2 <= r <= H-2, c <= W-2, which share no triangle and no
    vertex, so each flip is independent of the others; a flip replaces the
    edge by the one joining the two opposite triangle corners and is skipped
    when an endpoint would drop below degree 3.
    """
    if torus:
        if H < 3 or W < 3:
            raise ValueError("torus needs H, W >= 3")
        rr, cc = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        rr = rr.ravel()
        cc = cc.ravel()
        vid = lambda r, c: (r % H) * W + (c % W)  # noqa: E731
        hu, hv = vid(rr, cc), vid(rr, cc + 1)
        vu, vv = vid(rr, cc), vid(rr + 1, cc)
        qr, qc = rr, cc
    else:
        if H < 1 or W < 1:
            raise ValueError("grid needs H, W >= 1")
        vid = lambda r, c: r * W + c  # noqa: E731
        r1, c1 = np.meshgrid(np.arange(H), np.arange(W - 1), indexing="ij")
        hu, hv = vid(r1.ravel(), c1.ravel()), vid(r1.ravel(), c1.ravel() + 1)
        r2, c2 = np.meshgrid(np.arange(H - 1), np.arange(W), indexing="ij")
        vu, vv = vid(r2.ravel(), c2.ravel()), vid(r2.ravel() + 1, c2.ravel())
        r3, c3 = np.meshgrid(np.arange(H - 1), np.arange(W - 1), indexing="ij")
        qr, qc = r3.ravel(), c3.ravel()
    quad_id = qr * W + qc
    anti = (_mix64(seed, quad_id) & np.uint64(1)).astype(bool)
    du = np.where(anti, vid(qr, qc + 1), vid(qr, qc))
    dv = np.where(anti, vid(qr + 1, qc), vid(qr + 1, qc + 1))
    u = np.concatenate([hu, vu, du]).astype(np.int64)
    v = np.concatenate([hv, vv, dv]).astype(np.int64)

    if flip_frac > 0.0:
        n = H * W
        # eligible horizontal edges: even r in [2, H-2], even c in [0, W-2]
        er, ec = np.meshgrid(np.arange(2, H - 1, 2), np.arange(0, W - 1, 2), indexing="ij")
        er = er.ravel()
        ec = ec.ravel()
        if er.size:
            total_edges = u.size
            p = min(1.0, flip_frac * total_edges / er.size)
            hsh = _mix64(seed ^ 0x5DEECE66D, er * W + ec) >> np.uint64(11)
            pick = hsh.astype(np.float64) * (1.0 / float(1 << 53)) < p
            er, ec = er[pick], ec[pick]
            deg = np.bincount(np.concatenate([u, v]), minlength=n)
            a = vid(er, ec)
            b = vid(er, ec + 1)
            ok = (deg[a] > 3) & (deg[b] > 3)
            er, ec, a, b = er[ok], ec[ok], a[ok], b[ok]
            # opposite corner above: quad (r-1, c); below: quad (r, c)
            anti_up = (_mix64(seed, (er - 1) * W + ec) & np.uint64(1)).astype(bool)
            anti_dn = (_mix64(seed, er * W + ec) & np.uint64(1)).astype(bool)
            x = np.where(anti_up, vid(er - 1, ec + 1), vid(er - 1, ec))
            y = np.where(anti_dn, vid(er + 1, ec), vid(er + 1, ec + 1))
            # drop the flipped horizontal edges, add the new ones
            key_old = np.minimum(u, v) * n + np.maximum(u, v)
            key_rm = np.minimum(a, b) * n + np.maximum(a, b)
            keep = ~np.isin(key_old, key_rm)
            u = np.concatenate([u[keep], x]).astype(np.int64)
            v = np.concatenate([v[keep], y]).astype(np.int64)
    return u, v


def edges_to_csr(n: int, u: np.ndarray, v: np.ndarray, diag: bool = True,
                 index64: bool = False) -> CSR:
    """Symmetric pattern with sorted columns (duplicates removed)."""
    parts_r = [u, v]
    parts_c = [v, u]
    if diag:
        d = np.arange(n, dtype=np.int64)
        parts_r.append(d)
        parts_c.append(d)
    r = np.concatenate(parts_r).astype(np.int64)
    c = np.concatenate(parts_c).astype(np.int64)
    key = np.unique(r * n + c)
    r = key // n
    c = key % n
    counts = np.bincount(r, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if not index64:
        if rowptr[-1] >= 2**31:
            raise ValueError("nnz too large for int32 rowptr")
        rowptr = rowptr.astype(np.int32)
    return CSR(n, rowptr, c.astype(np.int32))


def grid_mesh(H: int, W: int, torus: bool, seed: int, flip_frac: float = 0.0,
              diag: bool = True, index64: bool = False) -> CSR:
    """Matrix pattern (vertex adjacency + diagonal) of a seeded grid/torus."""
    u, v = grid_edges(H, W, torus, seed, flip_frac)
    return edges_to_csr(H * W, u, v, diag=diag, index64=index64)


def grid_mesh_direct(H: int, W: int, torus: bool, seed: int, index64: bool = False) -> CSR:
    """Same pattern as ``grid_mesh(H, W, torus, seed)`` (no flips), built row
    by row from the grid geometry instead of from an edge list: each vertex
    lists itself, its axis neighbours and the diagonals of its four quads
    that pass through it.  Used where many large requests are generated."""
    if torus and (H < 3 or W < 3):
        raise ValueError("torus needs H, W >= 3")
    n = H * W
    r = np.repeat(np.arange(H, dtype=np.int64), W)
    c = np.tile(np.arange(W, dtype=np.int64), H)

    def vid(rr, cc):
        if torus:
            return (rr % H) * W + (cc % W), np.ones(rr.shape, dtype=bool)
        ok = (rr >= 0) & (rr < H) & (cc >= 0) & (cc < W)
        return np.where(ok, rr * W + cc, -1), ok

    bits = (_mix64(seed, np.arange(n, dtype=np.int64)) & np.uint64(1)).astype(bool)

    def quad(qr, qc):
        """(exists, anti-diagonal) of quad (qr, qc); quad ids are qr * W + qc."""
        if torus:
            qr, qc = qr % H, qc % W
            ok = np.ones(qr.shape, dtype=bool)
        else:
            ok = (qr >= 0) & (qr < H - 1) & (qc >= 0) & (qc < W - 1)
        return ok, bits[np.where(ok, qr * W + qc, 0)]

    cols = []
    for dr, dc in ((0, 0), (0, -1), (0, 1), (-1, 0), (1, 0)):
        v, ok = vid(r + dr, c + dc)
        cols.append(np.where(ok, v, -1))
    # quad above-left: diagonal (r-1,c-1)-(r,c) when not anti
    ok, anti = quad(r - 1, c - 1)
    v, vok = vid(r - 1, c - 1)
    cols.append(np.where(ok & ~anti & vok, v, -1))
    # quad below-right: (r,c)-(r+1,c+1) when not anti
    ok, anti = quad(r, c)
    v, vok = vid(r + 1, c + 1)
    cols.append(np.where(ok & ~anti & vok, v, -1))
    # quad above-right: (r-1,c+1)-(r,c) when anti
    ok, anti = quad(r - 1, c)
    v, vok = vid(r - 1, c + 1)
    cols.append(np.where(ok & anti & vok, v, -1))
    # quad below-left: (r,c)-(r+1,c-1) when anti
    ok, anti = quad(r, c - 1)
    v, vok = vid(r + 1, c - 1)
    cols.append(np.where(ok & anti & vok, v, -1))
    M = np.stack(cols, axis=1)
    M = np.where(M < 0, np.int64(1) << 62, M)
    M.sort(axis=1)
    keep = M < (np.int64(1) << 62)
    keep[:, 1:] &= M[:, 1:] != M[:, :-1]
    counts = keep.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colind = M[keep].astype(np.int32)
    if not index64:
        rowptr = rowptr.astype(np.int32)
    return CSR(n, rowptr, colind)


def block_expand(A: CSR, b: int, index64: bool = True) -> CSR:
    """Dense b x b block pattern: DOF b*k+r couples with DOF b*l+s iff A_kl != 0.

    Row DOF b*k+r lists, for each column l of row k (ascending), the b DOFs
    b*l .. b*l+b-1, so columns stay sorted.
    """
    n = A.n
    rp = A.rowptr.astype(np.int64)
    deg = np.diff(rp)
    nd = n * b
    row_len = np.repeat(deg * b, b)  # per DOF row
    rowptr = np.zeros(nd + 1, dtype=np.int64)
    np.cumsum(row_len, out=rowptr[1:])
    nnz = int(rowptr[-1])
    base = (A.colind.astype(np.int64) * b)
    # block row k: the expanded column list (length deg*b)
    exp_cols = (base[:, None] + np.arange(b, dtype=np.int64)[None, :]).ravel()
    blk_start = rp[:-1] * b
    colind = np.empty(nnz, dtype=np.int32)
    # each DOF row of block row k repeats exp_cols[blk_start[k] : blk_start[k]+deg[k]*b]
    for r in range(b):
        # destination offsets of DOF rows b*k + r
        dst = rowptr[np.arange(n) * b + r]
        idx = np.repeat(dst - blk_start, deg * b) + np.arange(exp_cols.size, dtype=np.int64)
        colind[idx] = exp_cols
    if not index64:
        if nnz >= 2**31:
            raise ValueError("nnz too large for int32 rowptr")
        rowptr = rowptr.astype(np.int32)
    return CSR(nd, rowptr, colind)


@dataclass
class MeshSpec:
    side: int
    torus: bool
    seed: int

    @property
    def n(self) -> int:
        return self.side * self.side


def batch_specs(seed: int, count: int = 256, smin: int = 45, smax: int = 447):
    """Side lengths log-uniform on [smin, smax] (n = side^2), torus/planar coin."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        s = int(round(math.exp(rng.uniform(math.log(smin), math.log(smax)))))
        torus = bool(rng.integers(0, 2))
        out.append(MeshSpec(s, torus, int(seed * 1000003 + i)))
    return out


def batch_meshes(seed: int, count: int = 256, smin: int = 45, smax: int = 447,
                 flip_frac: float = 0.05):
    return [grid_mesh(m.side, m.side, m.torus, m.seed, flip_frac) for m in
            batch_specs(seed, count, smin, smax)]


def concat_csr(meshes):
    """Concatenate CSRs with mesh-local column indices.

    Returns (rowptr64 over all rows with global nnz offsets, colind, vtx_off,
    nnz_off); each mesh's columns stay local to that mesh.
    """
    ns = [m.n for m in meshes]
    nz = [m.nnz for m in meshes]
    vtx_off = np.zeros(len(meshes) + 1, dtype=np.int64)
    nnz_off = np.zeros(len(meshes) + 1, dtype=np.int64)
    np.cumsum(ns, out=vtx_off[1:])
    np.cumsum(nz, out=nnz_off[1:])
    rowptr = np.zeros(int(vtx_off[-1]) + 1, dtype=np.int64)
    for i, m in enumerate(meshes):
        rowptr[vtx_off[i]:vtx_off[i + 1] + 1] = m.rowptr.astype(np.int64) + nnz_off[i]
    colind = np.concatenate([m.colind for m in meshes]).astype(np.int32)
    return rowptr, colind, vtx_off, nnz_off


def serving_stream(seed: int, count: int, rate: float = 200.0, smin: int = 100,
                   smax: int = 1414):
    """Poisson arrivals (exponential gaps, mean 1/rate s) of grid/torus requests.

    Returns a list of (arrival_time_s, MeshSpec); every request has its own
    diagonal seed.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        s = int(round(math.exp(rng.uniform(math.log(smin), math.log(smax)))))
        torus = bool(rng.integers(0, 2))
        out.append((t, MeshSpec(s, torus, int(seed * 7919 + i))))
    return out


def swap_quad_diagonals(A: CSR, W: int, quads) -> CSR:
    """The pattern of A (a grid or torus mesh of width W, vertex r*W + c)
    with the diagonal of each quad (r, c) moved to the other diagonal: the
    local pattern change of a remeshing step.  Indices wrap as on a torus.
    A quad whose first diagonal (r,c)-(r+1,c+1) is present gets the second
    one instead, and the other way round."""
    n = A.n
    H = n // W
    q = np.asarray(list(quads), dtype=np.int64).reshape(-1, 2)
    if len(q) == 0:
        return A
    r, c = q[:, 0], q[:, 1]

    def vid(rr, cc):
        return (rr % H) * W + (cc % W)

    a, b = vid(r, c), vid(r + 1, c + 1)
    x, y = vid(r, c + 1), vid(r + 1, c)
    rp = A.rowptr.astype(np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    key = rows * n + A.colind.astype(np.int64)
    has_ab = np.isin(a * n + b, key)
    old_u, old_v = np.where(has_ab, a, x), np.where(has_ab, b, y)
    new_u, new_v = np.where(has_ab, x, a), np.where(has_ab, y, b)
    drop = np.concatenate([old_u * n + old_v, old_v * n + old_u])
    key = key[~np.isin(key, drop)]
    key = np.unique(np.concatenate([key, new_u * n + new_v, new_v * n + new_u]))
    rr, cc = key // n, key % n
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rr, minlength=n), out=rowptr[1:])
    if A.rowptr.dtype == np.int32:
        rowptr = rowptr.astype(np.int32)
    return CSR(n, rowptr, cc.astype(np.int32))
