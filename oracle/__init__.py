"""ctypes binding of the serial CPU oracle (``fpo.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline leg of the benchmark may use this package; the GPU library never
does.  Every function takes host numpy arrays and returns host numpy arrays.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fpo.c")
_LIB_PATH = os.environ.get("FPO_LIB_PATH") or os.path.join(_HERE, "libfpo.so")
_lib = None

SCHED_LEVEL = 0
SCHED_POST = 1


def build(force: bool = True) -> str:
    """Compile fpo.c with gcc into oracle/libfpo.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC],
                       check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Opts(C.Structure):
    _fields_ = [("patch_size", C.c_int32), ("lloyd_iters", C.c_int32), ("seed", C.c_uint64),
                ("schedule", C.c_int32), ("block_size", C.c_int32), ("nd_level", C.c_int32),
                ("refine", C.c_int32), ("local_amd", C.c_int32)]


class _Out(C.Structure):
    _fields_ = [("perm", C.c_void_p), ("iperm", C.c_void_p), ("parent", C.c_void_p),
                ("colcount", C.c_void_p), ("nnzL", C.c_int64), ("gmap", C.c_void_p),
                ("node_of", C.c_void_p), ("node_begin", C.c_void_p), ("node_size", C.c_void_p),
                ("max_nodes", C.c_int32), ("n_patches", C.c_int32), ("depth", C.c_int32),
                ("n_nodes", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        vp = C.c_void_p
        L.fpo_mix64.restype = C.c_uint64
        L.fpo_mix64.argtypes = [C.c_uint64, C.c_uint64]
        L.fpo_graph_count.argtypes = [C.c_int64, vp, vp, C.c_int32, vp]
        L.fpo_graph_fill.argtypes = [C.c_int64, vp, vp, C.c_int32, vp, vp]
        L.fpo_patches.argtypes = [C.c_int32, vp, vp, C.c_int32, C.c_int32, C.c_uint64, vp, vp]
        L.fpo_grow.restype = C.c_int64
        L.fpo_grow.argtypes = [C.c_int32, vp, vp, C.c_int32, vp, vp]
        L.fpo_septree.argtypes = [C.c_int32, vp, vp, C.c_int32, vp, C.c_int32, C.c_int32, vp,
                                  vp, vp]
        L.fpo_bisect.argtypes = [C.c_int32, vp, vp, vp, vp]
        L.fpo_md.argtypes = [C.c_int32, vp, vp, vp]
        L.fpo_brute_md.argtypes = [C.c_int32, vp, vp, vp]
        L.fpo_amd.argtypes = [C.c_int32, vp, vp, vp, vp]
        L.fpo_etree.argtypes = [C.c_int32, vp, vp, vp, vp, vp]
        L.fpo_colcount.argtypes = [C.c_int32, vp, vp, vp, vp, vp, vp, vp]
        L.fpo_brute_symbolic.argtypes = [C.c_int32, vp, vp, vp, vp, vp, vp]
        L.fpo_supernodes.argtypes = [C.c_int32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.fpo_order.argtypes = [C.c_int64, vp, vp, vp, C.POINTER(_Opts), C.POINTER(_Out)]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")
    return rc


def mix64(seed: int, i: int) -> int:
    return int(lib().fpo_mix64(seed & 0xFFFFFFFFFFFFFFFF, i))


def graph(rowptr, colind, n_dof: int, block_size: int = 1):
    """O0: (g_rowptr int64, g_colind int32) of the vertex graph without diagonal."""
    rp = _i64(rowptr)
    ci = _i32(colind)
    nnz = np.zeros(1, dtype=np.int64)
    _check(lib().fpo_graph_count(n_dof, _p(rp), _p(ci), block_size, _p(nnz)), "graph_count")
    n_v = n_dof // block_size
    grp = np.zeros(n_v + 1, dtype=np.int64)
    gci = np.zeros(int(nnz[0]), dtype=np.int32)
    _check(lib().fpo_graph_fill(n_dof, _p(rp), _p(ci), block_size, _p(grp), _p(gci)), "graph_fill")
    return grp, gci


def patches(grp, gci, S: int, lloyd_iters: int = 1, seed: int = 0):
    """O1: (gmap, seeds) with P = len(seeds)."""
    n = len(grp) - 1
    grp = _i64(grp)
    gci = _i32(gci)
    gmap = np.zeros(n, dtype=np.int32)
    seeds = np.zeros(max(n, 1), dtype=np.int32)
    P = _check(lib().fpo_patches(n, _p(grp), _p(gci), S, lloyd_iters, seed & 0xFFFFFFFFFFFFFFFF,
                                 _p(gmap), _p(seeds)), "patches")
    return gmap, seeds[:P].copy()


def grow(grp, gci, seeds):
    n = len(grp) - 1
    grp = _i64(grp)
    gci = _i32(gci)
    seeds = _i32(seeds)
    label = np.zeros(n, dtype=np.int32)
    lib().fpo_grow(n, _p(grp), _p(gci), len(seeds), _p(seeds), _p(label))
    return label


def septree(grp, gci, gmap, P: int, nd_level: int = -1, refine: bool = False):
    """O2-O6: (node_of, pnode, D)."""
    n = len(grp) - 1
    grp = _i64(grp)
    gci = _i32(gci)
    gmap = _i32(gmap)
    node_of = np.zeros(n, dtype=np.int32)
    pnode = np.zeros(max(P, 1), dtype=np.int32)
    D = np.zeros(1, dtype=np.int32)
    _check(lib().fpo_septree(n, _p(grp), _p(gci), P, _p(gmap), nd_level, int(refine),
                             _p(node_of), _p(pnode), _p(D)), "septree")
    return node_of, pnode[:P].copy(), int(D[0])


def bisect(w, arp, aci):
    """O4 on a local quotient subgraph: boolean array, True = left child."""
    m = len(w)
    w = _i64(w)
    arp = _i64(arp)
    aci = _i32(aci)
    left = np.zeros(m, dtype=np.uint8)
    _check(lib().fpo_bisect(m, _p(w), _p(arp), _p(aci), _p(left)), "bisect")
    return left.astype(bool)


def md(rp, ci):
    m = len(rp) - 1
    rp = _i64(rp)
    ci = _i32(ci)
    order = np.zeros(max(m, 1), dtype=np.int32)
    _check(lib().fpo_md(m, _p(rp), _p(ci), _p(order)), "md")
    return order[:m].copy()


def amd(rp, ci, trace=False):
    """F3: approximate-minimum-degree order; with trace=True also the
    (m, m) array of approximate degrees at each pivot choice."""
    m = len(rp) - 1
    rp = _i64(rp)
    ci = _i32(ci)
    order = np.zeros(max(m, 1), dtype=np.int32)
    tr = np.zeros((m, m), dtype=np.int32) if trace else None
    _check(lib().fpo_amd(m, _p(rp), _p(ci), _p(order), _p(tr)), "amd")
    return (order[:m].copy(), tr) if trace else order[:m].copy()


def brute_md(rp, ci):
    m = len(rp) - 1
    rp = _i64(rp)
    ci = _i32(ci)
    order = np.zeros(max(m, 1), dtype=np.int32)
    _check(lib().fpo_brute_md(m, _p(rp), _p(ci), _p(order)), "brute_md")
    return order[:m].copy()


def etree(grp, gci, perm):
    n = len(grp) - 1
    perm = _i32(perm)
    iperm = np.empty(n, dtype=np.int32)
    iperm[perm] = np.arange(n, dtype=np.int32)
    parent = np.zeros(n, dtype=np.int32)
    _check(lib().fpo_etree(n, _p(_i64(grp)), _p(_i32(gci)), _p(perm), _p(iperm), _p(parent)),
           "etree")
    return parent


def colcount(grp, gci, perm, parent):
    n = len(grp) - 1
    perm = _i32(perm)
    iperm = np.empty(n, dtype=np.int32)
    iperm[perm] = np.arange(n, dtype=np.int32)
    cc = np.zeros(n, dtype=np.int32)
    nnz = np.zeros(1, dtype=np.int64)
    _check(lib().fpo_colcount(n, _p(_i64(grp)), _p(_i32(gci)), _p(perm), _p(iperm),
                              _p(_i32(parent)), _p(cc), _p(nnz)), "colcount")
    return cc, int(nnz[0])


def brute_symbolic(grp, gci, perm):
    n = len(grp) - 1
    parent = np.zeros(n, dtype=np.int32)
    cc = np.zeros(n, dtype=np.int32)
    nnz = np.zeros(1, dtype=np.int64)
    _check(lib().fpo_brute_symbolic(n, _p(_i64(grp)), _p(_i32(gci)), _p(_i32(perm)), _p(parent),
                                    _p(cc), _p(nnz)), "brute_symbolic")
    return parent, cc, int(nnz[0])


def supernodes(parent, colcount):
    """F1: fundamental supernodes of L from the elimination tree and column
    counts; returns a dict (Lp, super_of, super_ptr, super_parent, Lx_ptr,
    n_super)."""
    parent = _i32(parent)
    colcount = _i32(colcount)
    n = len(parent)
    Lp = np.zeros(n + 1, dtype=np.int64)
    sof = np.zeros(max(n, 1), dtype=np.int32)
    sptr = np.zeros(n + 1, dtype=np.int32)
    spar = np.zeros(max(n, 1), dtype=np.int32)
    lx = np.zeros(n + 1, dtype=np.int64)
    ns = np.zeros(1, dtype=np.int32)
    _check(lib().fpo_supernodes(n, _p(parent), _p(colcount), _p(Lp), _p(sof), _p(sptr), _p(spar),
                                _p(lx), _p(ns)), "supernodes")
    k = int(ns[0])
    return dict(Lp=Lp, super_of=sof[:n].copy(), super_ptr=sptr[:k + 1].copy(),
                super_parent=spar[:k].copy(), Lx_ptr=lx[:k + 1].copy(), n_super=k)


def order(rowptr, colind, n_dof: int, patch_size: int = 512, lloyd_iters: int = 1,
          seed: int = 0, schedule: int = SCHED_LEVEL, block_size: int = 1, user_gmap=None,
          nd_level: int = -1, refine: bool = False, local_amd: bool = False):
    """The whole ordering; returns a dict of numpy arrays and scalars."""
    rp = _i64(rowptr)
    ci = _i32(colind)
    n_v = n_dof // block_size
    opts = _Opts(patch_size, lloyd_iters, seed & 0xFFFFFFFFFFFFFFFF, schedule, block_size,
                 nd_level, int(refine), int(local_amd))
    perm = np.zeros(n_dof, dtype=np.int32)
    iperm = np.zeros(n_dof, dtype=np.int32)
    parent = np.zeros(n_dof, dtype=np.int32)
    cc = np.zeros(n_dof, dtype=np.int32)
    gmap = np.zeros(n_v, dtype=np.int32)
    node_of = np.zeros(n_v, dtype=np.int32)
    # capacity: D <= ceil(log2 n_v) + 1
    d = 0
    while (1 << d) < max(n_v, 1):
        d += 1
    cap = (1 << (d + 2)) - 1
    nb = np.zeros(cap, dtype=np.int32)
    ns = np.zeros(cap, dtype=np.int32)
    out = _Out(_p(perm).value, _p(iperm).value, _p(parent).value, _p(cc).value, 0,
               _p(gmap).value, _p(node_of).value, _p(nb).value, _p(ns).value, cap, 0, 0, 0)
    ug = None if user_gmap is None else _i32(user_gmap)
    _check(lib().fpo_order(n_dof, _p(rp), _p(ci), _p(ug), C.byref(opts), C.byref(out)), "order")
    nn = out.n_nodes
    return dict(perm=perm, iperm=iperm, parent=parent, colcount=cc, nnzL=int(out.nnzL),
                gmap=gmap, node_of=node_of, node_begin=nb[:nn].copy(), node_size=ns[:nn].copy(),
                P=int(out.n_patches), D=int(out.depth), n_nodes=int(nn))
