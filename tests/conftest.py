import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
# The mutation test points this at a directory holding an edited copy of the
# oracle package, so that the pins run against planted mistakes.
_ORACLE_COPY = os.environ.get("SCALP_ORACLE_COPY_ROOT")
if _ORACLE_COPY:
    sys.path.insert(0, _ORACLE_COPY)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    """The CPU oracle (built on first use if its library is absent)."""
    from oracle import oracle
    oracle.lib()
    return oracle
