import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


def pytest_terminal_summary(terminalreporter):
    """Repeat the GPU tests' result lines (errors against the oracle per
    multipole, batch and serving figures) after the run."""
    mod = sys.modules.get("tests.gpu_util")
    lines = getattr(mod, "REPORT", None) if mod is not None else None
    if lines:
        terminalreporter.section("GPU results against the oracle")
        for ln in lines:
            terminalreporter.write_line(ln)
