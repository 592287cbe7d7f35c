import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: statistical pins that take tens of seconds on the CPU")


def pytest_terminal_summary(terminalreporter):
    try:
        from tests.gpu_common import SUMMARY
    except Exception:
        return
    if SUMMARY:
        terminalreporter.write_sep("-", "parity: entries within rule T (1e-4 |orc| + 1e-7 max |orc|)")
        for line in SUMMARY:
            terminalreporter.write_line(line)
