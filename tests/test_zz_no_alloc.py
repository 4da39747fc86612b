"""The no-allocation batched launch (stencil_run_batched_noalloc) against the batched launch it
varies (stencil_run_batched, uncached), bit for bit, on two calls in a row, the second with a
smaller batch, with NaN-filled partner buffers; plus its size limit.  Collected last: it
shares the library's fixed scratch array with nothing else, and a failure here must not hide
the other tests of a run that stops at its first failure.
"""
import numpy as np
import pytest

import oracle
import paper_1802_00438_amd as S
from workloads import SETS, batch_grids

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _run_both(grids):
    x0s = [g.field() for g in grids]
    cfs = [SETS[g.coef_set] for g in grids]
    ts = [g.T for g in grids]
    ref = [torch.from_numpy(x).cuda() for x in x0s]
    S.stencil_run_batched(S._batch_items(ref, cfs, ts), None, None)  # uncached: synchronous
    got = [torch.from_numpy(x).cuda() for x in x0s]
    partners = [torch.full_like(x, float("nan")) for x in got]
    S.run_batched_noalloc(got, cfs, ts, partners)
    for i, (a, b) in enumerate(zip(got, ref)):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), i
    return x0s, cfs, ts, got


def test_noalloc_matches_batched_on_two_calls_second_smaller():
    big = batch_grids(n2d=8, n3d=4, lo2=100, hi2=1500, lo3=20, hi3=140, tlo=5, thi=90, seed=8800)
    small = batch_grids(n2d=3, n3d=2, lo2=30, hi2=300, lo3=6, hi3=50, tlo=1, thi=40, seed=8900)
    _run_both(big)
    x0s, cfs, ts, got = _run_both(small)
    # and the oracle, on the second call
    for x0, c, T, g in zip(x0s, cfs, ts, got):
        assert np.array_equal(g.cpu().numpy(), oracle.forward(x0, c, T, dtype=np.float32))


def test_noalloc_rejects_a_batch_beyond_its_scratch():
    # 40 grids of 2048^2 with 11200 steps: 700 passes of at least 40 tiles each, over 1.1e6
    # work items of 16 bytes, so the tables exceed 8 MiB; rejected before any device work
    xs = [torch.zeros((2048, 2048), device="cuda") for _ in range(40)]
    partners = [torch.zeros_like(x) for x in xs]
    with pytest.raises(S.StencilError) as ei:
        S.run_batched_noalloc(xs, [SETS["D2"]] * 40, [11200] * 40, partners)
    assert ei.value.status == -1
    assert "8388608" in str(ei.value)
