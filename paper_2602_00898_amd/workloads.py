"""Seeded workload recipes shared by the benchmark and the tests (inputs
only: sizes, seeds, patch targets; none of the ordering's arithmetic).

- batch: 256 grid/torus meshes, sides log-uniform on [45, 447], 5% edge
  flips, patch size from the committed autotune table, ordering seed
  3000 + i for mesh i;
- serving: Poisson arrivals at 200 requests/s, sides log-uniform on
  [100, 1414] (1e4 to 2e6 vertices), fresh diagonals per request, S = 512,
  ordering seed 7.
"""

from __future__ import annotations

from . import meshgen as mg

BATCH_SEED = 3
BATCH_FLIP = 0.05
SERVE_SEED = 5
SERVE_RATE = 200.0
SERVE_PATCH = 512
SERVE_ORDER_SEED = 7


def batch_order_seed(i: int) -> int:
    return BATCH_SEED * 1000 + i


def batch_patch_size(n: int) -> int:
    from .autotune import patch_size_for
    return patch_size_for(n)


def batch_mesh(spec):
    return mg.grid_mesh(spec.side, spec.side, spec.torus, spec.seed, BATCH_FLIP)


def batch_specs():
    return mg.batch_specs(BATCH_SEED)


def serving_stream(count: int):
    return mg.serving_stream(SERVE_SEED, count, rate=SERVE_RATE)


def serving_mesh(spec):
    return mg.grid_mesh_direct(spec.side, spec.side, spec.torus, spec.seed, index64=True)
