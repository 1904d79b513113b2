import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def ora():
    from oracle import oracle as O
    O.build()
    return O


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """Per-test parity-judge counts (elements judged, excused, failures), so
    that a quiet test run still records how many elements each test excused."""
    try:
        from tests.gpu_util import JUDGE_LOG
    except Exception:  # pragma: no cover - helper import failed; nothing judged
        return
    if not JUDGE_LOG:
        return
    tr = terminalreporter
    tr.section("parity judge: excused elements per test")
    for label, n, exc, fails, beyond, extra in JUDGE_LOG:
        tr.write_line("%-40s n=%-8d excused=%-5d (%.3f%%; %s; %d beyond horizon) failures=%d"
                      % (label, n, exc, 100.0 * exc / max(n, 1), extra, beyond, fails))
