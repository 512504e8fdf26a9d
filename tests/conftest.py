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
def c_oracle():
    from oracle import cgrid
    cgrid.build()
    return cgrid


@pytest.fixture(autouse=True)
def _clear_tuning_memo():
    """Each test starts from an empty tuning memo in the library (gr_autotune
    stores its winner there, and calls without a tuning read it)."""
    yield
    b = sys.modules.get("paper_1605_07023_amd.binding")
    if b is not None and getattr(b, "_lib", None) is not None:
        b._lib.gr_tuning_memo_clear()
