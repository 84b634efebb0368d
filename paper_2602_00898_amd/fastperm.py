"""Python binding of libfastperm.so (argument marshalling only).

Every step of the ordering runs in the HIP library; this module converts
torch device tensors to raw pointers, sizes the workspace through fp_query
and passes torch's current HIP stream.  It raises if the library is missing:
there is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import torch

from .build import LIB

SCHED_LEVEL = 0
SCHED_POST = 1

STATUS = {0: "ok", 1: "invalid argument", 2: "pattern not symmetric", 3: "index out of range",
          4: "workspace or device pool too small", 5: "out of device memory",
          6: "unsupported option", 7: "server busy", 8: "HIP runtime error",
          9: "device pipeline failure"}


class FpError(RuntimeError):
    def __init__(self, code, what, detail=None):
        msg = f"{what}: {STATUS.get(code, code)} (fp_status {code})"
        if detail:
            msg += " [device bits 0x%x, check %d, value %d]" % detail
        super().__init__(msg)
        self.code = code
        self.detail = detail


class Options(C.Structure):
    _fields_ = [("patch_size", C.c_int32), ("nd_level", C.c_int32), ("schedule", C.c_int32),
                ("block_size", C.c_int32), ("lloyd_iters", C.c_int32), ("seed", C.c_uint64),
                ("flags", C.c_uint32)]


class Csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr32", C.c_void_p),
                ("rowptr64", C.c_void_p), ("colind", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("perm", C.c_void_p), ("iperm", C.c_void_p), ("parent", C.c_void_p),
                ("colcount", C.c_void_p), ("nnzL", C.c_void_p), ("node_begin", C.c_void_p),
                ("node_size", C.c_void_p), ("gmap", C.c_void_p), ("n_nodes", C.c_void_p),
                ("status", C.c_void_p), ("max_nodes", C.c_int32)]


class SuperResult(C.Structure):
    _fields_ = [("Lp", C.c_void_p), ("super_ptr", C.c_void_p), ("n_super", C.c_void_p),
                ("super_of", C.c_void_p), ("super_parent", C.c_void_p), ("Lx_ptr", C.c_void_p),
                ("status", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("md_lds_bytes", C.c_int32), ("md_blocks_per_cu", C.c_int32),
                ("max_lds_bytes", C.c_int32)]


class HostCsr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("colind", C.c_void_p)]


_lib = None


def lib():
    """Load libfastperm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is missing: build it with paper_2602_00898_amd.build.build()")
        L = C.CDLL(LIB)
        vp = C.c_void_p
        L.fp_version.restype = C.c_int
        L.fp_status_str.restype = C.c_char_p
        L.fp_status_str.argtypes = [C.c_int]
        L.fp_options_default.argtypes = [C.POINTER(Options)]
        L.fp_options_default.restype = None
        L.fp_create.argtypes = [C.POINTER(vp)]
        L.fp_destroy.argtypes = [vp]
        L.fp_query.argtypes = [vp, C.POINTER(Csr), C.POINTER(Options), C.POINTER(C.c_size_t),
                               C.POINTER(C.c_int32)]
        L.fp_order.argtypes = [vp, C.POINTER(Csr), vp, C.POINTER(Options), vp, C.c_size_t,
                               C.POINTER(Result), vp]
        L.fp_order_static.argtypes = [vp, C.POINTER(Csr), vp, C.POINTER(Options),
                                      C.POINTER(Result), vp]
        L.fp_order_update.argtypes = [vp, C.POINTER(Csr), vp, vp, C.POINTER(Options), vp,
                                      C.c_size_t, C.POINTER(Result), vp, vp]
        L.fp_last_error.argtypes = [vp, vp, vp]
        L.fp_error_detail.argtypes = [vp, vp, vp, C.POINTER(C.c_uint32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32)]
        L.fp_stage_count.restype = C.c_int
        L.fp_stage_name.restype = C.c_char_p
        L.fp_stage_name.argtypes = [C.c_int]
        L.fp_stage_times.argtypes = [vp, C.POINTER(C.c_float), C.c_int32]
        L.fp_time_kernel.argtypes = [vp, C.c_char_p]
        L.fp_kernel_time.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_int32)]
        L.fp_query_batch.argtypes = [vp, C.c_int32, C.POINTER(Csr), C.POINTER(Options),
                                     C.POINTER(vp), C.POINTER(C.c_size_t), C.POINTER(C.c_int32)]
        L.fp_order_batch.argtypes = [vp, C.c_int32, C.POINTER(Csr), C.POINTER(vp),
                                     C.POINTER(Options), vp, C.c_size_t, C.POINTER(Result), vp]
        i64p = C.POINTER(C.c_int64)
        L.fp_query_batch_concat.argtypes = [vp, C.c_int32, vp, vp, i64p, i64p, C.POINTER(Options),
                                            C.POINTER(C.c_size_t), i64p]
        L.fp_order_batch_concat.argtypes = [vp, C.c_int32, vp, vp, i64p, i64p, C.POINTER(Options),
                                            vp, C.c_size_t, vp, vp, vp, vp, vp, vp, vp, vp, i64p,
                                            vp]
        L.fp_server_create.argtypes = [vp, C.c_size_t, C.c_int32, C.POINTER(vp)]
        L.fp_server_submit.argtypes = [vp, C.POINTER(HostCsr), C.POINTER(Options),
                                       C.POINTER(C.c_uint64)]
        L.fp_server_test.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int32)]
        L.fp_server_wait.argtypes = [vp, C.c_uint64, vp, vp, vp, vp, C.POINTER(C.c_int64),
                                     C.POINTER(C.c_double)]
        L.fp_server_destroy.argtypes = [vp]
        L.fp_graph_create.argtypes = [vp, C.c_int32, vp, vp, vp, vp, C.c_size_t, vp,
                                      C.POINTER(C.c_void_p)]
        L.fp_graph_launch.argtypes = [vp, vp]
        L.fp_graph_destroy.argtypes = [vp]
        L.fp_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.fp_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.fp_supernodes_query.argtypes = [C.c_int64, C.POINTER(C.c_size_t)]
        L.fp_supernodes.argtypes = [vp, C.c_int64, vp, vp, vp, C.c_size_t,
                                    C.POINTER(SuperResult), vp]
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check(rc, what):
    if rc != 0:
        raise FpError(rc, what)


class Handle:
    """fp_handle bound to the current device, with a reusable workspace."""

    def __init__(self):
        h = C.c_void_p()
        _check(lib().fp_create(C.byref(h)), "fp_create")
        self.h = h
        self._ws = None

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.fp_destroy(self.h)
            self.h = None

    def tuning(self):
        """(md_lds_bytes, md_blocks_per_cu, max_lds_bytes) of this handle."""
        t = Tuning()
        _check(lib().fp_get_tuning(self.h, C.byref(t)), "fp_get_tuning")
        return t.md_lds_bytes, t.md_blocks_per_cu, t.max_lds_bytes

    def set_tuning(self, md_lds_bytes, md_blocks_per_cu):
        t = Tuning(int(md_lds_bytes), int(md_blocks_per_cu), 0)
        _check(lib().fp_set_tuning(self.h, C.byref(t)), "fp_set_tuning")

    def workspace(self, nbytes, device):
        if self._ws is None or self._ws.numel() < nbytes or self._ws.device != device:
            self._ws = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        return self._ws


FLAG_TIMING = 1
FLAG_VALIDATE = 2
FLAG_REFINE = 4
FLAG_AMD = 8


def options(patch_size=512, schedule=SCHED_LEVEL, block_size=1, lloyd_iters=1, seed=0,
            flags=FLAG_VALIDATE, nd_level=-1):
    o = Options()
    lib().fp_options_default(C.byref(o))
    o.patch_size = patch_size
    o.nd_level = nd_level
    o.schedule = schedule
    o.block_size = block_size
    o.lloyd_iters = lloyd_iters
    o.seed = seed & 0xFFFFFFFFFFFFFFFF
    o.flags = flags
    return o


def _mesh_options(m):
    """Options of one matrix of a batch or graph from its dict (keys
    patch_size, schedule, block_size, lloyd_iters, seed, nd_level, refine,
    flags)."""
    flags = (m.get("flags", FLAG_VALIDATE) | (FLAG_REFINE if m.get("refine") else 0)
             | (FLAG_AMD if m.get("amd") else 0))
    return options(m.get("patch_size", 512), m.get("schedule", SCHED_LEVEL), m.get("block_size", 1),
                   m.get("lloyd_iters", 1), m.get("seed", 0), flags, m.get("nd_level", -1))


def make_csr(n, rowptr, colind):
    c = Csr()
    c.n = n
    c.nnz = int(colind.numel())
    if rowptr.dtype == torch.int32:
        c.rowptr32 = rowptr.data_ptr()
    else:
        c.rowptr64 = rowptr.data_ptr()
    c.colind = colind.data_ptr() if colind.numel() else None
    return c


def query(handle, n, rowptr, colind, opts):
    A = make_csr(n, rowptr, colind)
    ws = C.c_size_t()
    mx = C.c_int32()
    _check(lib().fp_query(handle.h, C.byref(A), C.byref(opts), C.byref(ws), C.byref(mx)),
           "fp_query")
    return ws.value, mx.value


def order(rowptr, colind, n, *, patch_size=512, schedule=SCHED_LEVEL, block_size=1,
          lloyd_iters=1, seed=0, user_gmap=None, handle=None, out=None, stream=None,
          check=True, timing=False, validate=True, nd_level=-1, refine=False, amd=False):
    """Order one matrix on the GPU.  rowptr (int32/int64) and colind (int32)
    are device tensors.  Returns a dict of device tensors; with check=True
    the call synchronises and raises on device-reported errors.  validate
    checks on the device that the pattern is symmetric; nd_level limits the
    tree depth (-1: full); refine selects minimum-cover separators; amd
    approximate-minimum-degree local orders."""
    dev = colind.device if colind.numel() else rowptr.device
    handle = handle or Handle()
    opts = options(patch_size, schedule, block_size, lloyd_iters, seed,
                   (FLAG_TIMING if timing else 0) | (FLAG_VALIDATE if validate else 0)
                   | (FLAG_REFINE if refine else 0) | (FLAG_AMD if amd else 0), nd_level)
    A = make_csr(n, rowptr, colind)
    ws_bytes, max_nodes = query(handle, n, rowptr, colind, opts)
    ws = handle.workspace(ws_bytes, dev)
    if out is None:
        i32 = dict(dtype=torch.int32, device=dev)
        out = dict(perm=torch.empty(n, **i32), iperm=torch.empty(n, **i32),
                   parent=torch.empty(n, **i32), colcount=torch.empty(n, **i32),
                   nnzL=torch.zeros(1, dtype=torch.int64, device=dev),
                   node_begin=torch.empty(max_nodes, **i32), node_size=torch.empty(max_nodes, **i32),
                   gmap=torch.empty(max(n // block_size, 1), **i32),
                   n_nodes=torch.zeros(1, **i32), status=torch.zeros(1, dtype=torch.int32, device=dev))
    R = Result(_ptr(out["perm"]), _ptr(out["iperm"]), _ptr(out["parent"]), _ptr(out["colcount"]),
               _ptr(out["nnzL"]), _ptr(out.get("node_begin")), _ptr(out.get("node_size")),
               _ptr(out.get("gmap")), _ptr(out.get("n_nodes")), _ptr(out.get("status")),
               int(out["node_begin"].numel()) if out.get("node_begin") is not None else 0)
    s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
    rc = lib().fp_order(handle.h, C.byref(A), _ptr(user_gmap), C.byref(opts), _ptr(ws),
                        ws_bytes, C.byref(R), C.c_void_p(s))
    if rc != 0:
        device_side = rc in (3, 4, 9)
        raise FpError(rc, "fp_order", error_detail(handle, ws, s) if device_side else None)
    if check:
        rc = lib().fp_last_error(handle.h, _ptr(ws), C.c_void_p(s))
        if rc != 0:
            raise FpError(rc, "device", error_detail(handle, ws, s))
    return out


def supernodes(parent, colcount, *, handle=None, stream=None, check=True):
    """Fundamental supernodes of L from an ordering's parent and colcount
    (int32 device tensors of n entries) through fp_supernodes.  Returns a
    dict of device tensors: Lp, super_ptr, n_super, super_of, super_parent,
    Lx_ptr, status (super_ptr / super_parent / Lx_ptr hold capacity n+1;
    their first n_super(+1) entries are written)."""
    n = int(parent.numel())
    dev = parent.device
    handle = handle or Handle()
    ws_bytes = C.c_size_t()
    _check(lib().fp_supernodes_query(n, C.byref(ws_bytes)), "fp_supernodes_query")
    ws = torch.empty(max(int(ws_bytes.value), 1), dtype=torch.uint8, device=dev)
    i32 = dict(dtype=torch.int32, device=dev)
    out = dict(Lp=torch.empty(n + 1, dtype=torch.int64, device=dev),
               super_ptr=torch.empty(n + 1, **i32), n_super=torch.zeros(1, **i32),
               super_of=torch.empty(max(n, 1), **i32), super_parent=torch.empty(max(n, 1), **i32),
               Lx_ptr=torch.empty(n + 1, dtype=torch.int64, device=dev),
               status=torch.zeros(1, **i32))
    R = SuperResult(*[_ptr(out[k]) for k in ("Lp", "super_ptr", "n_super", "super_of",
                                              "super_parent", "Lx_ptr", "status")])
    s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
    _check(lib().fp_supernodes(handle.h, n, _ptr(parent), _ptr(colcount), _ptr(ws),
                               ws_bytes.value, C.byref(R), C.c_void_p(s)), "fp_supernodes")
    out["_ws"] = ws  # the workspace lives until the results are read
    if check:
        torch.cuda.synchronize(dev)
        if int(out["status"].item()):
            raise FpError(9, "fp_supernodes: parent array is not an elimination tree")
    return out


def order_update(rowptr, colind, n, prev_gmap, prev_workspace, *, patch_size=512,
                 schedule=SCHED_LEVEL, block_size=1, lloyd_iters=1, seed=0, handle=None, out=None,
                 stream=None, check=True):
    """fp_order_update: order a changed pattern on the same vertices keeping
    an earlier call's patches (prev_gmap, its gmap output) and reusing the
    local orders of unchanged nodes from its workspace (prev_workspace, a
    device tensor that must not be the workspace of `handle`).  Returns the
    output dict plus 'reused' (vertices whose local order was reused)."""
    dev = colind.device if colind.numel() else rowptr.device
    handle = handle or Handle()
    opts = options(patch_size, schedule, block_size, lloyd_iters, seed)
    A = make_csr(n, rowptr, colind)
    ws_bytes, max_nodes = query(handle, n, rowptr, colind, opts)
    ws = handle.workspace(ws_bytes, dev)
    if ws.data_ptr() == prev_workspace.data_ptr():
        raise ValueError("order_update needs a workspace other than the earlier call's")
    if out is None:
        out = _alloc_out(n, max_nodes, block_size, dev)
    out["reused"] = torch.zeros(1, dtype=torch.int32, device=dev)
    R = _result(out)
    s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
    rc = lib().fp_order_update(handle.h, C.byref(A), _ptr(prev_gmap), _ptr(prev_workspace),
                               C.byref(opts), _ptr(ws), ws_bytes, C.byref(R), _ptr(out["reused"]),
                               C.c_void_p(s))
    if rc != 0:
        raise FpError(rc, "fp_order_update")
    if check:
        rc = lib().fp_last_error(handle.h, _ptr(ws), C.c_void_p(s))
        if rc != 0:
            raise FpError(rc, "device", error_detail(handle, ws, s))
    return out


def order_static(rowptr, colind, n, *, patch_size=512, schedule=SCHED_LEVEL, block_size=1,
                 lloyd_iters=1, seed=0, user_gmap=None, handle=None, out=None, stream=None,
                 check=True):
    """order() through fp_order_static: the library's static device scratch
    instead of a workspace (the call allocates nothing itself)."""
    dev = colind.device if colind.numel() else rowptr.device
    handle = handle or Handle()
    opts = options(patch_size, schedule, block_size, lloyd_iters, seed)
    A = make_csr(n, rowptr, colind)
    if out is None:
        _, max_nodes = query(handle, n, rowptr, colind, opts)
        out = _alloc_out(n, max_nodes, block_size, dev)
    R = _result(out)
    s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
    rc = lib().fp_order_static(handle.h, C.byref(A), _ptr(user_gmap), C.byref(opts), C.byref(R),
                               C.c_void_p(s))
    if rc != 0:
        raise FpError(rc, "fp_order_static")
    if check:
        torch.cuda.synchronize(dev)
        bits = int(out["status"].item())
        if bits:
            raise FpError(9, "device", (bits, 0, 0))
    return out


def error_detail(handle, ws, stream=0):
    """(device error bits, first failing check, its value) of the last call."""
    bits, site, arg = C.c_uint32(), C.c_int32(), C.c_int32()
    rc = lib().fp_error_detail(handle.h, _ptr(ws), C.c_void_p(stream), C.byref(bits),
                               C.byref(site), C.byref(arg))
    return None if rc != 0 else (bits.value, site.value, arg.value)


def stage_times(handle):
    """Per-stage device milliseconds of the handle's last timed call."""
    L = lib()
    k = L.fp_stage_count()
    ms = (C.c_float * k)()
    _check(L.fp_stage_times(handle.h, ms, k), "fp_stage_times")
    return {L.fp_stage_name(i).decode(): float(ms[i]) for i in range(k)}


def _alloc_out(n, max_nodes, block_size, dev):
    i32 = dict(dtype=torch.int32, device=dev)
    return dict(perm=torch.empty(n, **i32), iperm=torch.empty(n, **i32),
                parent=torch.empty(n, **i32), colcount=torch.empty(n, **i32),
                nnzL=torch.zeros(1, dtype=torch.int64, device=dev),
                node_begin=torch.empty(max_nodes, **i32), node_size=torch.empty(max_nodes, **i32),
                gmap=torch.empty(max(n // block_size, 1), **i32),
                n_nodes=torch.zeros(1, **i32), status=torch.zeros(1, dtype=torch.int32, device=dev))


def _result(out):
    return Result(_ptr(out["perm"]), _ptr(out["iperm"]), _ptr(out["parent"]), _ptr(out["colcount"]),
                  _ptr(out["nnzL"]), _ptr(out["node_begin"]), _ptr(out["node_size"]),
                  _ptr(out["gmap"]), _ptr(out["n_nodes"]), _ptr(out["status"]),
                  int(out["node_begin"].numel()))


def order_batch(meshes, *, handle=None, stream=None, check=True, outs=None):
    """Order many matrices in one call (fp_order_batch).  `meshes` is a list
    of dicts with device tensors rowptr, colind, the size n and optional
    patch_size, seed, schedule, block_size, lloyd_iters, nd_level, refine,
    amd, user_gmap.  Returns one output dict per matrix, as order() does;
    `outs` (the list an earlier call on the same matrices returned) is
    reused instead of allocating new outputs."""
    L = lib()
    k = len(meshes)
    handle = handle or Handle()
    if k == 0:
        return []
    A = (Csr * k)()
    O = (Options * k)()
    R = (Result * k)()
    G = (C.c_void_p * k)()
    keep = []
    for i, m in enumerate(meshes):
        A[i] = make_csr(m["n"], m["rowptr"], m["colind"])
        O[i] = _mesh_options(m)
        ug = m.get("user_gmap")
        G[i] = None if ug is None else ug.data_ptr()
        keep.append(ug)
    ws, mx = C.c_size_t(), C.c_int32()
    _check(L.fp_query_batch(handle.h, k, A, O, G, C.byref(ws), C.byref(mx)), "fp_query_batch")
    dev = meshes[0]["colind"].device
    reuse = outs is not None
    if reuse and len(outs) != k:
        raise ValueError("outs must hold one output dict per matrix")
    outs = list(outs) if reuse else []
    for i, m in enumerate(meshes):
        if reuse:
            if outs[i]["perm"].numel() != m["n"] or outs[i]["node_begin"].numel() < mx.value:
                raise ValueError(f"outs[{i}] does not fit matrix {i}")
        else:
            outs.append(_alloc_out(m["n"], mx.value, m.get("block_size", 1), dev))
        R[i] = _result(outs[i])
    wbuf = handle.workspace(ws.value, dev)
    s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
    rc = L.fp_order_batch(handle.h, k, A, G, O, _ptr(wbuf), ws.value, R, C.c_void_p(s))
    if rc != 0:
        raise FpError(rc, "fp_order_batch")
    if check:
        torch.cuda.synchronize(dev)
        st = torch.cat([o["status"] for o in outs]).cpu()
        bad = torch.nonzero(st).flatten().tolist()
        if bad:
            raise FpError(9, f"fp_order_batch: matrix {bad[0]} device bits 0x{int(st[bad[0]]):x}")
    return outs


def order_batch_concat(rowptr, colind, vtx_off, nnz_off, opts_list, *, handle=None, stream=None,
                       check=True):
    """fp_order_batch_concat: concatenated per-mesh CSR (rowptr int64 device
    tensor holding each mesh's n_i+1 local row pointers, colind int32 device
    tensor with local column indices; vtx_off / nnz_off host sequences of
    n_mesh+1 offsets).  opts_list: one dict of options per mesh.  Returns a
    dict of concatenated device tensors (perm, iperm, parent, colcount at the
    vertex offsets; nnzL and status per mesh; node_begin/node_size at
    node_off) and node_off itself."""
    import numpy as np
    L = lib()
    k = len(opts_list)
    handle = handle or Handle()
    O = (Options * k)()
    for i, o in enumerate(opts_list):
        O[i] = _mesh_options(o)
    vo = np.ascontiguousarray(vtx_off, dtype=np.int64)
    no = np.ascontiguousarray(nnz_off, dtype=np.int64)
    node_off = np.zeros(k + 1, dtype=np.int64)
    i64p = C.POINTER(C.c_int64)
    ws = C.c_size_t()
    _check(L.fp_query_batch_concat(handle.h, k, _ptr(rowptr), _ptr(colind),
                                   vo.ctypes.data_as(i64p), no.ctypes.data_as(i64p), O,
                                   C.byref(ws), node_off.ctypes.data_as(i64p)),
           "fp_query_batch_concat")
    dev = rowptr.device
    ntot = int(vo[-1])
    i32 = dict(dtype=torch.int32, device=dev)
    out = dict(perm=torch.empty(ntot, **i32), iperm=torch.empty(ntot, **i32),
               parent=torch.empty(ntot, **i32), colcount=torch.empty(ntot, **i32),
               nnzL=torch.zeros(k, dtype=torch.int64, device=dev), status=torch.zeros(k, **i32),
               node_begin=torch.empty(int(node_off[-1]), **i32),
               node_size=torch.empty(int(node_off[-1]), **i32))
    wbuf = handle.workspace(ws.value, dev)
    s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
    rc = L.fp_order_batch_concat(handle.h, k, _ptr(rowptr), _ptr(colind),
                                 vo.ctypes.data_as(i64p), no.ctypes.data_as(i64p), O, _ptr(wbuf),
                                 ws.value, _ptr(out["perm"]), _ptr(out["iperm"]),
                                 _ptr(out["parent"]), _ptr(out["colcount"]), _ptr(out["nnzL"]),
                                 _ptr(out["status"]), _ptr(out["node_begin"]),
                                 _ptr(out["node_size"]), node_off.ctypes.data_as(i64p),
                                 C.c_void_p(s))
    if rc != 0:
        raise FpError(rc, "fp_order_batch_concat")
    out["node_off"] = node_off
    if check:
        torch.cuda.synchronize(dev)
        st = out["status"].cpu()
        bad = torch.nonzero(st).flatten().tolist()
        if bad:
            raise FpError(9, f"fp_order_batch_concat: matrix {bad[0]} device bits "
                             f"0x{int(st[bad[0]]):x}")
    return out


class Graph:
    """A recorded ordering (fp_graph_create): one matrix or a batch, replayed
    by launch() with one host call.  `meshes` as for order_batch.  The
    output dicts (`outputs`, one per matrix) are written by every replay;
    the input tensors are read anew by every replay (same n and nnz)."""

    def __init__(self, meshes, *, handle=None):
        L = lib()
        k = len(meshes)
        if k == 0:
            raise ValueError("Graph needs at least one matrix")
        self.handle = handle or Handle()
        A = (Csr * k)()
        O = (Options * k)()
        R = (Result * k)()
        G = (C.c_void_p * k)()
        self._keep = []
        for i, m in enumerate(meshes):
            A[i] = make_csr(m["n"], m["rowptr"], m["colind"])
            O[i] = _mesh_options(m)
            ug = m.get("user_gmap")
            G[i] = None if ug is None else ug.data_ptr()
            self._keep += [m["rowptr"], m["colind"], ug]
        ws, mx = C.c_size_t(), C.c_int32()
        _check(L.fp_query_batch(self.handle.h, k, A, O, G, C.byref(ws), C.byref(mx)),
               "fp_query_batch")
        dev = meshes[0]["colind"].device
        self.device = dev
        self.outputs = []
        for i, m in enumerate(meshes):
            self.outputs.append(_alloc_out(m["n"], mx.value, m.get("block_size", 1), dev))
            R[i] = _result(self.outputs[i])
        # the graph's own workspace (it must outlive the graph)
        self.workspace = torch.empty(int(ws.value), dtype=torch.uint8, device=dev)
        torch.cuda.synchronize(dev)
        g = C.c_void_p()
        _check(L.fp_graph_create(self.handle.h, k, A, G, O, _ptr(self.workspace), ws.value, R,
                                 C.byref(g)), "fp_graph_create")
        self.g = g

    def launch(self, stream=None, check=False):
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().fp_graph_launch(self.g, C.c_void_p(s)), "fp_graph_launch")
        if check:
            torch.cuda.synchronize(self.device)
            st = torch.cat([o["status"] for o in self.outputs]).cpu()
            bad = torch.nonzero(st).flatten().tolist()
            if bad:
                raise FpError(9, f"graph replay: matrix {bad[0]} device bits "
                                 f"0x{int(st[bad[0]]):x}")
        return self.outputs

    def __del__(self):
        if getattr(self, "g", None) is not None and _lib is not None:
            torch.cuda.synchronize(self.device)
            _lib.fp_graph_destroy(self.g)
            self.g = None


class Server:
    """Request server (fp_server_*): host CSR in, host results out."""

    def __init__(self, hbm_budget, max_slots, handle=None):
        self.handle = handle or Handle()
        s = C.c_void_p()
        _check(lib().fp_server_create(self.handle.h, int(hbm_budget), int(max_slots), C.byref(s)),
               "fp_server_create")
        self.s = s
        self._keep = {}

    def submit(self, rowptr, colind, n, **kw):
        import numpy as np
        rp = np.ascontiguousarray(rowptr, dtype=np.int64)
        ci = np.ascontiguousarray(colind, dtype=np.int32)
        A = HostCsr(n, ci.size, rp.ctypes.data, ci.ctypes.data if ci.size else None)
        o = options(kw.get("patch_size", 512), kw.get("schedule", SCHED_LEVEL),
                    kw.get("block_size", 1), kw.get("lloyd_iters", 1), kw.get("seed", 0))
        t = C.c_uint64()
        _check(lib().fp_server_submit(self.s, C.byref(A), C.byref(o), C.byref(t)),
               "fp_server_submit")
        self._keep[t.value] = (rp, ci, n)
        return t.value

    def test(self, ticket):
        d = C.c_int32()
        _check(lib().fp_server_test(self.s, ticket, C.byref(d)), "fp_server_test")
        return bool(d.value)

    def wait(self, ticket):
        import numpy as np
        n = self._keep[ticket][2]
        r = {k: np.empty(n, np.int32) for k in ("perm", "iperm", "parent", "colcount")}
        nz, lat = C.c_int64(), C.c_double()
        rc = lib().fp_server_wait(self.s, ticket, r["perm"].ctypes.data, r["iperm"].ctypes.data,
                                  r["parent"].ctypes.data, r["colcount"].ctypes.data,
                                  C.byref(nz), C.byref(lat))
        self._keep.pop(ticket, None)
        if rc != 0:
            raise FpError(rc, "fp_server_wait")
        r["nnzL"] = nz.value
        r["latency_s"] = lat.value
        return r

    def close(self):
        if getattr(self, "s", None) is not None and _lib is not None:
            _lib.fp_server_destroy(self.s)
            self.s = None
            self._keep.clear()

    def __del__(self):
        self.close()


def time_kernel(handle, name):
    """Time every launch of kernel `name` in later calls on `handle`."""
    _check(lib().fp_time_kernel(handle.h, (name or "").encode()), "fp_time_kernel")


def kernel_time(handle):
    """(total ms, launches) of the timed kernel in the handle's last call."""
    ms, k = C.c_float(), C.c_int32()
    _check(lib().fp_kernel_time(handle.h, C.byref(ms), C.byref(k)), "fp_kernel_time")
    return ms.value, k.value
