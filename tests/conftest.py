import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU oracle check")


@pytest.fixture(scope="session")
def params():
    from workloads import default_params
    return default_params()


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """Measured parity figures (errors against their bounds, directions compared), one line each."""
    try:
        from tests.gpu_util import format_records
    except ImportError:
        return
    lines = format_records()
    if lines:
        terminalreporter.write_sep("-", "parity records")
        for line in lines:
            terminalreporter.write_line(line)
