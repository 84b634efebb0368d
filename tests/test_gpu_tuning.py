"""GPU: execution settings of the local-order stage change speed only.

The local order of a node is a function of the node's induced subgraph
(Sec. 4.3, Step 4); the LDS a workgroup gives it and the number of
workgroups per CU decide only where and when it runs (in LDS or, past the
dense layout's size, in the global pool).  So every tuning an autotuner may
pick must give the oracle's result, single and batched.
"""

import pytest

from tests.gpu_util import compare, cpu_order, gpu_order, mesh, say

pytestmark = pytest.mark.gpu

# (md_lds_bytes, md_blocks_per_cu): smallest LDS (most nodes in the pool),
# the default, the whole LDS; one to eight workgroups per CU
TUNINGS = [(16 * 1024, 1), (64 * 1024, 2), (96 * 1024, 4), (None, 8)]
CASES = [(40, 40, True, 31, 0.05, 64), (96, 80, False, 32, 0.05, 256), (128, 128, True, 33, 0.05, 512)]


def _tuned_handle(lds, per_cu):
    from paper_2602_00898_amd import fastperm as fpm
    h = fpm.Handle()
    big = h.tuning()[2]
    h.set_tuning(big if lds is None else min(lds, big), per_cu)
    got = h.tuning()
    assert got[0] == (big if lds is None else min(lds, big)) and got[1] == per_cu
    return h


@pytest.mark.parametrize("lds,per_cu", TUNINGS)
def test_single_under_tuning(lds, per_cu):
    h = _tuned_handle(lds, per_cu)
    for H, W, t, s, f, S in CASES:
        A = mesh(H, W, t, s, f)
        say(f"[tuning] lds={lds} per_cu={per_cu} {H}x{W} S={S}")
        compare(gpu_order(A, patch_size=S, seed=s, handle=h), cpu_order(A, patch_size=S, seed=s),
                f"tuning {lds}/{per_cu} {H}x{W}")


@pytest.mark.parametrize("lds,per_cu", [TUNINGS[0], TUNINGS[3]])
def test_batch_under_tuning(lds, per_cu):
    import torch

    from paper_2602_00898_amd import fastperm as fpm
    from tests.test_gpu_batch import MIX, _device_meshes, _to_dict
    h = _tuned_handle(lds, per_cu)
    cases = [(mesh(H, W, t, s, f), S, s) for H, W, t, s, f, S in MIX]
    say(f"[tuning] batch lds={lds} per_cu={per_cu}")
    outs = fpm.order_batch(_device_meshes(cases), handle=h)
    torch.cuda.synchronize()
    for (A, S, s), out in zip(cases, outs):
        compare(_to_dict(out, A), cpu_order(A, patch_size=S, seed=s), f"batch tuned n={A.n}")


def test_invalid_tuning_refused():
    from paper_2602_00898_amd import fastperm as fpm
    h = fpm.Handle()
    before = h.tuning()
    big = before[2]
    for lds, per_cu in [(8 * 1024, 2), (big + 1024, 2), (64 * 1024 + 4, 2), (64 * 1024, 0),
                        (64 * 1024, 9)]:
        with pytest.raises(fpm.FpError):
            h.set_tuning(lds, per_cu)
    assert h.tuning() == before
