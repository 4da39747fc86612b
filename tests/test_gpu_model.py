"""The library's time model of a plan (stencil_plan_model) follows the plan's resolved blocking.

The model itself is a heuristic used to rank tuning candidates, so its accuracy is measured
(bench.py, `model_accuracy`) rather than asserted; these tests pin what it must report
exactly: the pass count of the blocking and the split into memory and arithmetic parts.
"""
import math

import pytest

import paper_1802_00438_amd as S
from workloads import HOTSPOT, HOTSPOT_PHYS, DIFFUSION

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("form,shape,tuning", [
    (HOTSPOT, (512, 700), {"variant": 2, "k": 12, "seg_len": 64}),
    (HOTSPOT_PHYS, (512, 700), {"variant": 2, "k": 8, "seg_len": 64}),
    (DIFFUSION, (300, 301), {"variant": 2, "k": 16, "seg_len": 50}),
    (DIFFUSION, (40, 70, 130), {"variant": 2, "k": 3}),
    (HOTSPOT, (20, 64, 200), {"variant": 2, "k": 2, "seg_len": 10}),
])
def test_plan_model_follows_the_blocking(form, shape, tuning):
    plan = S.Plan(form, shape, tuning)
    try:
        k = plan.tuning["k"]
        assert k == tuning["k"]
        for T in (0, 1, k, 5 * k + 1, 1000):
            m = plan.model(T)
            assert m["passes"] == math.ceil(T / k)
            assert m["mem_seconds"] >= 0 and m["alu_seconds"] >= 0
            # each pass costs the larger of its two parts plus a launch overhead
            assert m["seconds"] >= max(m["mem_seconds"], m["alu_seconds"]) - 1e-15
            assert m["seconds"] <= m["mem_seconds"] + m["alu_seconds"] + 1e-5 * m["passes"] + 1e-15
        with pytest.raises(S.StencilError):
            plan.model(-1)
    finally:
        plan.close()


def test_plan_model_of_the_plain_kernel():
    plan = S.Plan(HOTSPOT, (256, 512), {"variant": 1})
    try:
        m = plan.model(37)
        assert m["passes"] == 37 and m["alu_seconds"] == 0.0
        # every step moves the grid in, the power map in and the grid out once
        one = plan.model(1)
        assert abs(m["mem_seconds"] - 37 * one["mem_seconds"]) <= 1e-12
    finally:
        plan.close()


@pytest.mark.parametrize("r,k", [(2, 4), (3, 2), (4, 1)])
def test_plan_model_of_star_plans(r, k):
    plan = S.StarPlan(r, (300, 700), {"variant": 2, "k": k, "seg_len": 64})
    try:
        for T in (0, 1, k, 7 * k + 1):
            m = plan.model(T)
            assert m["passes"] == math.ceil(T / k)
            assert m["seconds"] >= max(m["mem_seconds"], m["alu_seconds"]) - 1e-15
    finally:
        plan.close()
