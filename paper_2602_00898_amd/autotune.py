"""Patch-size table for batched ordering.

The target patch size S is an input of the ordering (it changes the result),
so the batch takes S from a fixed table indexed by mesh size.  `tune()`
measures, on the current GPU, the ordering time of a seeded torus mesh per
size bucket for each S in {128, 256, 512, 1024} and keeps the fastest; the
table it writes (`tune_table.json` beside this file) is what
`patch_size_for` reads.  Without a table the defaults below apply.

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


def patch_size_for(n: int) -> int:
    """Patch size of a mesh with n vertices from the table."""
    t = load()
    for bound, s in zip(t["bounds"], t["patch_size"]):
        if n < bound:
            return int(s)
    return int(t["patch_size"][-1])


def tune(reps: int = 3, verbose: bool = True) -> dict:
    import torch

    from . import fastperm as fpm
    from . import meshgen as mg

    dev = torch.device("cuda:0")
    h = fpm.Handle()
    chosen, timings = [], {}
    for bound, side in BUCKETS:
        A = mg.grid_mesh(side, side, True, 7, 0.05)
        rp = torch.from_numpy(A.rowptr).to(dev)
        ci = torch.from_numpy(A.colind).to(dev)
        best, best_t = None, None
        for S in CANDIDATES:
            fpm.order(rp, ci, A.n, patch_size=S, seed=7, handle=h)  # warm
            torch.cuda.synchronize(dev)
            ts = []
            for _ in range(reps):
                t = time.perf_counter()
                fpm.order(rp, ci, A.n, patch_size=S, seed=7, handle=h)
                torch.cuda.synchronize(dev)
                ts.append(time.perf_counter() - t)
            t_med = sorted(ts)[len(ts) // 2]
            timings[f"{side}x{side}/S={S}"] = round(t_med * 1e3, 3)
            if verbose:
                print(f"[tune] {side}x{side} S={S}: {t_med * 1e3:.2f} ms", flush=True)
            if best_t is None or t_med < best_t:
                best, best_t = S, t_med
        chosen.append(best)
    table = {"bounds": [b for b, _ in BUCKETS], "patch_size": chosen, "ms": timings,
             "device": torch.cuda.get_device_name(dev)}
    with open(TABLE, "w") as f:
        json.dump(table, f, indent=1)
    global _table
    _table = table
    return table


if __name__ == "__main__":
    print(json.dumps(tune()))
