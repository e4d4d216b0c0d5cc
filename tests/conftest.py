import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a HIP device (runs on the MI355X box)")
    config.addinivalue_line("markers", "slow: longer CPU checks of the oracle")


def pytest_addoption(parser):
    parser.addoption("--runslow", action="store_true", default=False,
                     help="also run the tests marked slow (long CPU checks of the oracle)")


def pytest_collection_modifyitems(config, items):
    import pytest
    if config.getoption("--runslow") or os.environ.get("PDG_RUN_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow: run with --runslow")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)
