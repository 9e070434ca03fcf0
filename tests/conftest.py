import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as O
    O.lib()
    return O


def pytest_terminal_summary(terminalreporter):
    """Every bounded parity comparison of the run, with its error and bound."""
    try:
        from tests.gpu_helpers import BOUNDS
    except Exception:
        return
    if not BOUNDS:
        return
    tr = terminalreporter
    tr.section("parity errors and their bounds")
    for test, what, err, bound in BOUNDS:
        tr.write_line(f"{err:9.2e} <= {bound:9.2e}  {what}  [{test}]")
