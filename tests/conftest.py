import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; runs the HIP library")


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


# Per-workload error of the FP32 GPU result against the FP64 oracle, filled by
# test_gpu_fp64_report.py and printed at the end of the session.
FP64_REPORT = []


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    if not FP64_REPORT:
        return
    terminalreporter.write_sep("-", "FP32 GPU result vs FP64 oracle, per workload")
    for name, what, err, note in FP64_REPORT:
        terminalreporter.write_line("%-24s %-34s max-rel %.3e  %s" % (name, what, err, note))
