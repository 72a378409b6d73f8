import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
# tests/test_oracle_mutants.py runs the oracle's pins against a copy of the
# oracle package with one planted mistake: that copy is imported instead
_ORACLE_COPY = os.environ.get("DRTS_ORACLE_COPY")
if _ORACLE_COPY:
    sys.path.insert(0, _ORACLE_COPY)
    import oracle  # noqa: E402,F401  (cached now, so later imports get the copy)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    if _ORACLE_COPY:
        assert os.path.abspath(oracle.__file__).startswith(os.path.abspath(_ORACLE_COPY))
    oracle.build()
    return oracle
