"""Error paths of the batched launch, forced from the host.

A dependency wait of the persistent kernels is bounded.  With STENCIL_DEBUG_SPIN_LIMIT=0 every
wait that is not satisfied at its first poll gives up at once: the launch still runs to its
end (every item is computed, on whatever its inputs hold, and every index stays inside its
grid), and the library must report STENCIL_ERR_INTERNAL rather than a result.  A launch
without the override must then be bit-exact again.
"""
import numpy as np
import pytest

import oracle
import paper_1802_00438_amd as S
from workloads import SETS, uniform

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _batch():
    # one grid with far more items per pass than it takes to start them, so that pass-1 items
    # are claimed while their pass-0 neighbours still run
    x0 = uniform((2048, 2048), 0.0, 1.0, 9100)
    return x0, SETS["D2"], 64


def test_bounded_wait_reports_internal_error_uncached(monkeypatch):
    x0, cf, T = _batch()
    x = torch.from_numpy(x0).cuda()
    monkeypatch.setenv("STENCIL_DEBUG_SPIN_LIMIT", "0")
    with pytest.raises(S.StencilError) as ei:
        S.stencil_run_batched(S._batch_items([x], [cf], [T]), None, None)
    assert ei.value.status == -5
    torch.cuda.synchronize()
    monkeypatch.delenv("STENCIL_DEBUG_SPIN_LIMIT")
    x.copy_(torch.from_numpy(x0))
    S.stencil_run_batched(S._batch_items([x], [cf], [T]), None, None)
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), oracle.forward(x0, cf, T, dtype=np.float32))


def test_bounded_wait_reported_by_batch_sync(monkeypatch):
    x0, cf, T = _batch()
    x = torch.from_numpy(x0).cuda()
    monkeypatch.setenv("STENCIL_DEBUG_SPIN_LIMIT", "0")
    cache = S.run_batched([x], [cf], [T])  # captured with the override
    monkeypatch.delenv("STENCIL_DEBUG_SPIN_LIMIT")
    try:
        with pytest.raises(S.StencilError) as ei:
            S.stencil_batch_sync(cache)
        assert ei.value.status == -5
        # the flag is sticky: a later replay reports it too once the earlier one is done
        with pytest.raises(S.StencilError):
            S.run_batched([x], [cf], [T], cache=cache)
    finally:
        S.stencil_batch_destroy(cache)
    # a batch captured without the override is exact and reports OK
    x.copy_(torch.from_numpy(x0))
    cache = S.run_batched([x], [cf], [T])
    try:
        S.stencil_batch_sync(cache)
        assert np.array_equal(x.cpu().numpy(), oracle.forward(x0, cf, T, dtype=np.float32))
    finally:
        S.stencil_batch_destroy(cache)
