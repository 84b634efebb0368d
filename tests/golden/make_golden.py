"""Writes the oracle regression fixtures in this folder.

Calls only the CPU oracle and the input generators.  Run from the repository
root:  python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2602_00898_amd import meshgen as mg  # noqa: E402

CASES = {
    # name: (H, W, torus, mesh seed, flip, S, method seed, schedule, block)
    "torus6x6_S8": (6, 6, True, 21, 0.0, 8, 21, oracle.SCHED_LEVEL, 1),
    "planar9x7_S5_post": (9, 7, False, 22, 0.0, 5, 22, oracle.SCHED_POST, 1),
    "planar64x64_S64": (64, 64, False, 1, 0.0, 64, 1, oracle.SCHED_LEVEL, 1),
    "torus48x48_flip_S128": (48, 48, True, 23, 0.05, 128, 23, oracle.SCHED_LEVEL, 1),
    "torus8x8_block3_S6": (8, 8, True, 24, 0.0, 6, 24, oracle.SCHED_LEVEL, 3),
}


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


def run(case):
    H, W, torus, ms, flip, S, seed, sched, b = case
    A = mg.grid_mesh(H, W, torus, ms, flip)
    if b > 1:
        A = mg.block_expand(A, b)
    return oracle.order(A.rowptr, A.colind, A.n, patch_size=S, seed=seed, schedule=sched,
                        block_size=b)


def main():
    out = {}
    for name, case in CASES.items():
        r = run(case)
        e = dict(case=list(case), nnzL=r["nnzL"], P=r["P"], D=r["D"])
        for k in ("perm", "parent", "colcount", "gmap", "node_of", "node_begin", "node_size"):
            e[k + "_sha256"] = digest(r[k])
        if len(r["perm"]) <= 200:
            for k in ("perm", "parent", "colcount", "gmap"):
                e[k] = [int(x) for x in r[k]]
        out[name] = e
    with open(os.path.join(HERE, "oracle_fixtures.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
