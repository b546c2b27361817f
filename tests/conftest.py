import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: longer CPU checks")


def pytest_terminal_summary(terminalreporter):
    """Prints every parity run's compared-track count and excuses."""
    pu = sys.modules.get("parity_util")
    tallies = getattr(pu, "SESSION_TALLIES", [])
    if tallies:
        terminalreporter.write_sep("-", "parity excuses per run (margin / diverged / FP64 referee)")
        for t in tallies:
            terminalreporter.write_line(t.line())
