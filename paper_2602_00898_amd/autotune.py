"""Autotune table: patch size per mesh size, and execution settings.

The target patch size S is an input of the ordering (it changes the result),
so a batch takes S from a fixed table indexed by mesh size.  The execution
settings of the local-order stage (LDS per workgroup, workgroups per CU;
`Handle.set_tuning`) change speed only, never a result.

`tune()` measures on the current GPU, per size bucket, the ordering time of
a seeded torus mesh (5% edge flips) for each S in {128, 256, 512, 1024} and
keeps the fastest; then, with that S, the time under each execution
setting of `EXEC_GRID`, summed over the same torus with and without the
flips and taken on calls queued back to back; then the same settings on a
seeded batch of mixed meshes.  The
table it writes (`tune_table.json` beside this file) is what
`patch_size_for`, `exec_for` and `exec_batch` read.  Without a table the
defaults below apply.

    python -m paper_2602_00898_amd.autotune      # on a GPU: rewrite the table
"""

from __future__ import annotations

import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tune_table.json")
CANDIDATES = (128, 256, 512, 1024)
# bucket upper bounds (vertices) and the side of the torus that stands for it
BUCKETS = ((8192, 64), (32768, 128), (131072, 256), (524288, 512), (1 << 31, 1024))
DEFAULT = {"bounds": [b for b, _ in BUCKETS], "patch_size": [128, 256, 512, 512, 512]}
# (LDS bytes per local-order workgroup, workgroups per CU); None = the whole LDS
EXEC_GRID = tuple((lds, per_cu) for lds in (32 * 1024, 64 * 1024, 96 * 1024, None)
                  for per_cu in (1, 2, 4))
# the batch the execution settings are tuned on: 48 seeded meshes, sides
# log-uniform on [45, 447] (the batch workload's recipe, fewer meshes)
TUNE_BATCH = 48

_table = None


def load():
    global _table
    if _table is None:
        try:
            with open(TABLE) as f:
                _table = json.load(f)
        except (OSError, ValueError):
            _table = DEFAULT
    return _table


def _bucket(n: int) -> int:
    t = load()
    for i, bound in enumerate(t["bounds"]):
        if n < bound:
            return i
    return len(t["bounds"]) - 1


def patch_size_for(n: int) -> int:
    """Patch size of a mesh with n vertices from the table."""
    return int(load()["patch_size"][_bucket(n)])


def exec_for(n: int):
    """(md_lds_bytes, md_blocks_per_cu) for ordering one mesh of n vertices,
    or None (library defaults).  An LDS of 0 stands for the whole LDS."""
    e = load().get("exec_single")
    return None if not e else tuple(e[_bucket(n)])


def exec_batch():
    """(md_lds_bytes, md_blocks_per_cu) for batched orderings, or None."""
    e = load().get("exec_batch")
    return None if not e else tuple(e)


def apply(handle, setting) -> None:
    """Set a table entry on a Handle (None leaves the handle as it is)."""
    if setting is None:
        return
    lds, per_cu = setting
    big = handle.tuning()[2]
    handle.set_tuning(big if not lds else min(int(lds), big), int(per_cu))


def _queued_ms(fn, sync, reps, k=8):
    """Median over reps of the time per call of k calls queued back to back
    (one synchronisation each), as an application ordering many matrices in
    a row sees them."""
    fn()
    sync()
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        for _ in range(k):
            fn()
        sync()
        ts.append((time.perf_counter() - t) / k)
    return sorted(ts)[len(ts) // 2] * 1e3


def _median_ms(fn, sync, reps):
    fn()
    sync()
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        sync()
        ts.append(time.perf_counter() - t)
    return sorted(ts)[len(ts) // 2] * 1e3


def tune(reps: int = 3, verbose: bool = True) -> dict:
    import torch

    from . import fastperm as fpm
    from . import meshgen as mg

    dev = torch.device("cuda:0")

    def sync():
        torch.cuda.synchronize(dev)

    def say(s):
        if verbose:
            print(f"[tune] {s}", flush=True)

    h = fpm.Handle()
    default = h.tuning()[:2]
    chosen, timings, exec_single = [], {}, []
    for bound, side in BUCKETS:
        A = mg.grid_mesh(side, side, True, 7, 0.05)
        rp = torch.from_numpy(A.rowptr).to(dev)
        ci = torch.from_numpy(A.colind).to(dev)
        h.set_tuning(*default)
        best = None
        for S in CANDIDATES:
            ms = _median_ms(lambda: fpm.order(rp, ci, A.n, patch_size=S, seed=7, handle=h), sync,
                            reps)
            timings[f"{side}x{side}/S={S}"] = round(ms, 3)
            say(f"{side}x{side} S={S}: {ms:.2f} ms")
            if best is None or ms < best[1]:
                best = (S, ms)
        S = best[0]
        chosen.append(S)
        # execution settings: summed over the same torus with and without the
        # edge flips (separators of degree-5/7 meshes and of plain ones load
        # the local orders differently), calls queued on resident outputs
        B = mg.grid_mesh(side, side, True, 7, 0.0)
        rpB = torch.from_numpy(B.rowptr).to(dev)
        ciB = torch.from_numpy(B.colind).to(dev)
        outA = fpm.order(rp, ci, A.n, patch_size=S, seed=7, handle=h)
        outB = fpm.order(rpB, ciB, B.n, patch_size=S, seed=7, handle=h)
        sync()
        best_e = None
        for lds, per_cu in EXEC_GRID:
            apply(h, (lds, per_cu))
            ms = sum(_queued_ms(lambda: fpm.order(r_, c_, n_, patch_size=S, seed=7, handle=h, out=o_,
                                                  check=False), sync, reps)
                     for r_, c_, n_, o_ in ((rp, ci, A.n, outA), (rpB, ciB, B.n, outB)))
            timings[f"{side}x{side}/S={S}/lds={lds or 0}/cu={per_cu}"] = round(ms, 3)
            say(f"{side}x{side} S={S} lds={lds or 'all'} per_cu={per_cu}: {ms:.2f} ms")
            if best_e is None or ms < best_e[1]:
                best_e = ((lds or 0, per_cu), ms)
        exec_single.append(list(best_e[0]))
    global _table
    _table = {"bounds": [b for b, _ in BUCKETS], "patch_size": chosen}
    specs = mg.batch_specs(3)[:TUNE_BATCH]
    meshes = [mg.grid_mesh(s.side, s.side, s.torus, s.seed, 0.05) for s in specs]
    dm = [dict(rowptr=torch.from_numpy(A.rowptr).to(dev), colind=torch.from_numpy(A.colind).to(dev),
               n=A.n, patch_size=patch_size_for(A.n), seed=3000 + i) for i, A in enumerate(meshes)]
    hb = fpm.Handle()
    best_b = None
    for lds, per_cu in EXEC_GRID:
        apply(hb, (lds, per_cu))
        ms = _median_ms(lambda: fpm.order_batch(dm, handle=hb), sync, reps)
        timings[f"batch{TUNE_BATCH}/lds={lds or 0}/cu={per_cu}"] = round(ms, 3)
        say(f"batch of {TUNE_BATCH} lds={lds or 'all'} per_cu={per_cu}: {ms:.2f} ms")
        if best_b is None or ms < best_b[1]:
            best_b = ((lds or 0, per_cu), ms)
    table = {"bounds": [b for b, _ in BUCKETS], "patch_size": chosen,
             "exec_single": exec_single, "exec_batch": list(best_b[0]), "ms": timings,
             "device": torch.cuda.get_device_name(dev)}
    with open(TABLE, "w") as f:
        json.dump(table, f, indent=1)
    _table = table
    return table


if __name__ == "__main__":
    print(json.dumps(tune()))
