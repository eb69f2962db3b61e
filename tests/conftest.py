import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def golden_path(name):
    return os.path.join(ROOT, "tests", "golden", name)


def read_table(name):
    rows = []
    with open(golden_path(name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


def pytest_terminal_summary(terminalreporter):
    """Largest per-particle err/tol ratio of every element-wise parity check that ran."""
    import sys
    mod = sys.modules.get("elementwise")
    ratios = getattr(mod, "RATIOS", None) if mod else None
    if not ratios:
        return
    terminalreporter.write_sep("-", "element-wise parity: largest err/tol per check")
    for name, r in ratios:
        terminalreporter.write_line(f"{r:9.3g}  {name}")
